"""Build libchw.so in-tree with hipcc for gfx950.

Every HIP translation unit is compiled with the packed-FP32 feature turned off
and without fast-math (the stage order fixes the rounding; reassociation must
not change it).  Translation units compile in parallel.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchw.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++20", "-fPIC", "-fno-fast-math", "-Wall",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [
    "chw_kernels_f32.hip",
    "chw_kernels_bf16.hip",
    "chw_kernels_f16.hip",
    "chw_kernels_i32.hip",
    "chw_kernels_f64.hip",
    "chw_philox.hip",
    "chw_nodes.hip",
    "chw_scratch.hip",
    "chw_registry.cpp",
    "chw_planner.cpp",
    "chw_api.cpp",
    "chw_selfcheck.cpp",
    "chw_plancheck.cpp",
]


# Host-side sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer) for the
# CPU checks of the planner, plan checker, layout self-check and argument
# validation: every flag applies to the host compilation only (the device code
# is built as usual, without them).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
SAN_LIB = os.path.join(HERE, "libchw_san.so")
SAN_DIR = os.path.join(HERE, "_build", "san")


def _compile(src, sanitize=False):
    out_dir = SAN_DIR if sanitize else BUILD_DIR
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += DEVICE
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    if sanitize:
        cmd += SANITIZE
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), "\n".join(msgs)))
    return obj


def build(verbose=False, jobs=None):
    """Compile every source and link libchw.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


def build_sanitized(verbose=False, jobs=None):
    """Host-only libchw_san.so with ASan and UBSan (see SANITIZE).  A Python
    process loads it with the sanitizer runtime preloaded
    (sanitizer_runtime()) and CHW_LIBRARY pointing at it."""
    os.makedirs(SAN_DIR, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize=True), SOURCES))
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-shared-libsan", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB, file=sys.stderr)
    return SAN_LIB


def sanitizer_runtime():
    """Path of the compiler's shared ASan runtime (to LD_PRELOAD into Python)."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        res = subprocess.run([HIPCC, "--print-runtime-dir"], capture_output=True, text=True)
        path = os.path.join(res.stdout.strip(), "libclang_rt.asan-x86_64.so")
    return path


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitize":
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
