"""Build the gfx950 HIP library libfbsde.so in-tree (hipcc, no torch extension machinery).

Usage: python -m paper_2510_02635_amd.build  [-q] [--host-sanitize]

--host-sanitize builds a second copy, _lib/hostsan/libfbsde.so, whose host code (argument checks,
workspace carving, tile plans, schedules, caches) carries AddressSanitizer and UndefinedBehaviorSanitizer
instrumentation; the device code is the same.  `python -m paper_2510_02635_amd.hostsan` runs tests against it.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libfbsde.so")
SOURCES = ["fbsde_api.hip", "fbsde_shared_api.hip", "fbsde_batched_api.hip", "fbsde_literal.hip", "fbsde_sigma.hip"]
ARCH = "gfx950"

# Packed FP32 instructions are switched off for every HIP translation unit: the kernels are
# written with scalar / float2 FP32 code and must not be turned into v_pk_* forms.
HIPCC_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm toolchain required to build libfbsde.so)")
    return exe


# Host-only sanitizers: each -fsanitize applies to the host pass alone (the device code is not instrumented).
HOSTSAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOSTSAN_LIB = os.path.join(LIBDIR, "hostsan", "libfbsde.so")


def build(verbose=True, host_sanitize=False):
    from concurrent.futures import ThreadPoolExecutor
    libdir = os.path.dirname(HOSTSAN_LIB) if host_sanitize else LIBDIR
    lib = HOSTSAN_LIB if host_sanitize else LIB
    extra = HOSTSAN_FLAGS if host_sanitize else []
    os.makedirs(libdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(libdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as pool:
        results = list(pool.map(lambda j: subprocess.run(j[0], capture_output=True, text=True), jobs))
    for (cmd, _), res in zip(jobs, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise subprocess.CalledProcessError(res.returncode, cmd)
        if verbose and res.stderr:
            # hipcc's host pass does not know the packed-FP32 target feature: drop that note
            lines = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
            if lines:
                sys.stderr.write("\n".join(lines) + "\n")
    objs = [obj for _, obj in jobs]
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *[f for f in extra if f != "-g"], *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv, host_sanitize="--host-sanitize" in sys.argv)
