"""Run tests against the host-sanitized library (AddressSanitizer + UndefinedBehaviorSanitizer on the host
code; build it with `python -m paper_2510_02635_amd.build --host-sanitize`).

Usage: python -m paper_2510_02635_amd.hostsan [pytest arguments]   (default: the CPU tests that call the
library: tests/test_abi.py, tests/test_batched_plan.py, tests/test_host_sizes.py)

Host code only: the ROCm AddressSanitizer runtime also intercepts the HSA device-memory calls for device-side
checking, which needs XNACK, so a process that allocates device memory under it fails at its first allocation.

The interpreter is not instrumented, so the sanitizer runtime is preloaded into a child pytest process;
leak checking is off (the interpreter and the HIP runtime keep allocations until exit) and the first
report ends the run with a non-zero status.
"""
import os
import subprocess
import sys

from . import build as B


def asan_runtime():
    clang = os.path.join(os.path.dirname(os.path.realpath(B.hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if out.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the AddressSanitizer runtime of the ROCm clang was not found")
    return path


def main(argv):
    if not os.path.exists(B.HOSTSAN_LIB):
        sys.stderr.write(f"{B.HOSTSAN_LIB} is missing: python -m paper_2510_02635_amd.build --host-sanitize\n")
        return 2
    env = dict(os.environ)
    env["FBSDE_LIB_PATH"] = B.HOSTSAN_LIB
    # the sanitizer runtime must come first; whatever the environment already preloads stays after it
    env["LD_PRELOAD"] = ":".join([asan_runtime()] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    args = argv or [os.path.join(B.ROOT, "tests", t) for t in ("test_abi.py", "test_batched_plan.py", "test_host_sizes.py")]
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *args]
    print("hostsan:", " ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=B.ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
