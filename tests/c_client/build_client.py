"""Builds the plain C client the GPU tests run (sphint_client.c beside this file): gcc, the
public header and the HIP runtime API only, linked against the built libsphint.so.

    python tests/c_client/build_client.py      (also part of __graft_entry__.build())
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2510_09892_amd")
EXE = os.path.join(HERE, "sphint_client")


def build(verbose: bool = False) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler (gcc) for the C client")
    if not os.path.exists(os.path.join(PKG, "libsphint.so")):
        raise RuntimeError("libsphint.so is not built (python -m paper_2510_09892_amd.build)")
    cmd = [cc, "-O2", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(rocm, 'include')}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(HERE, "sphint_client.c"), "-o", EXE + ".tmp", f"-L{PKG}", "-lsphint",
           f"-L{os.path.join(rocm, 'lib')}", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2510_09892_amd", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C client build failed:\n{r.stdout}{r.stderr}")
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
