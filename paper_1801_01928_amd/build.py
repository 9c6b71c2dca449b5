"""Builds libttgfx.so (every HIP source under csrc/) for gfx950 with hipcc.

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file, where the binding loads it.  ``--asan`` (or
build(asan=True)) also builds libttgfx_asan.so: the same sources with the
host code instrumented by AddressSanitizer (device code unchanged), loaded
by the CPU tests of the C ABI's validation and bookkeeping under the ASan
runtime.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libttgfx.so")
ASAN_LIB = os.path.join(HERE, "libttgfx_asan.so")
ARCH = os.environ.get("TTGFX_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every device pass.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Wall",
          "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC] + DEVICE_FLAGS


# host-only AddressSanitizer: every sanitizer flag applies to the host pass
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime():
    """Path of the ASan runtime the instrumented library needs preloaded."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], stdout=subprocess.PIPE,
                         text=True).stdout.strip()
    return out if out and os.path.exists(out) else None


def _compile(src, asan=False):
    obj = os.path.join(BUILD, "asan" if asan else "", os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + (ASAN_HOST if asan else []) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False, jobs=None, asan=False):
    os.makedirs(os.path.join(BUILD, "asan") if asan else BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda src: _compile(src, asan), srcs))
    for obj, out in results:
        if verbose and out.strip():
            print(out)
    objs = [o for o, _ in results]
    lib = ASAN_LIB if asan else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + (ASAN_HOST if asan else []) + ["-o", tmp] + objs
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, asan="--asan" in sys.argv))
