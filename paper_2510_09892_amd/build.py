"""Build libsphint.so (gfx950 HIP) and the CPU test build of its per-pair arithmetic.

    python -m paper_2510_09892_amd.build

Flags: -ffp-contract=off keeps the compiler from fusing a*b+c into FMAs the error-free
transformations do not ask for (the paper builds with the same flag, Sec. 7.2); packed FP32
instructions are disabled for all device code.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsphint.so")
HOSTCHECK = os.path.join(PKG, "libsphint_hostcheck.so")
ARCH = os.environ.get("SPHINT_ARCH", "gfx950")

DEVICE_SOURCES = ["sphint.hip", "sphint_batch.hip", "sphint_cand.hip", "sphint_arcarc.hip",
                  "sphint_adaptive.hip", "sphint_ablation.hip"]
COMMON = ["-O3", "-fPIC", "-shared", "-std=c++17", "-ffp-contract=off",
          f"-I{INCLUDE}", f"-I{CSRC}"]


def _hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libsphint)")


def _clang():
    c = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
    if os.path.exists(c):
        return c
    raise RuntimeError("ROCm clang++ not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in line and line.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build failed ({' '.join(cmd)}):\n{out}")
    if out and verbose:
        print(out)


def build(verbose: bool = False) -> str:
    """Compile both libraries; returns the path of libsphint.so."""
    srcs = [os.path.join(CSRC, s) for s in DEVICE_SOURCES]
    tmp = LIB + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", *COMMON,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          *srcs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    tmp = HOSTCHECK + ".tmp"
    _run([_clang(), "-x", "hip", "--cuda-host-only", *COMMON,
          os.path.join(CSRC, "sphint_hostcheck.cpp"), "-o", tmp], verbose)
    os.replace(tmp, HOSTCHECK)
    return LIB


def build_hostcheck_sanitized(out: str, verbose: bool = False) -> str:
    """The CPU test build under AddressSanitizer and UndefinedBehaviorSanitizer (host code
    only; no GPU code is involved).  Load it with the sanitizer runtime preloaded:

        LD_PRELOAD=$(python -m paper_2510_09892_amd.build --asan-runtime) \
        ASAN_OPTIONS=detect_leaks=0 SPHINT_HOSTCHECK_LIB=<out> python -m pytest tests/...
    """
    _run([_clang(), "-x", "hip", "--cuda-host-only", *COMMON, "-O1", "-g",
          "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address,undefined",
          "-Xarch_host", "-fno-sanitize-recover=undefined", "-shared-libsan",
          os.path.join(CSRC, "sphint_hostcheck.cpp"), "-o", out], verbose)
    return out


def asan_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime (for LD_PRELOAD)."""
    r = subprocess.run([_clang(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    if "--asan-runtime" in sys.argv:
        print(asan_runtime())
    elif "--sanitized" in sys.argv:
        print(build_hostcheck_sanitized(sys.argv[sys.argv.index("--sanitized") + 1],
                                        verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
