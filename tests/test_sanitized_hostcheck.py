"""The CPU build of the kernel arithmetic under AddressSanitizer and UndefinedBehaviorSanitizer.

The exact expansion arithmetic indexes fixed-size buffers (the arena the GPU keeps in LDS is a
plain array in the host build), and the candidate rule does binary searches over the
latitude table: the host-build tests (hit rule, ties, exact fallbacks, candidates, arc x arc,
adaptive bounds, formula replicas) run again in a child process against a build with both
sanitizers, which aborts on the first finding.  Host code only; nothing runs on a GPU.
"""

import os
import subprocess
import sys

import pytest

from paper_2510_09892_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["tests/test_hostcheck.py", "tests/test_hostcheck_ablation.py",
         "tests/test_hostcheck_adaptive.py", "tests/test_hostcheck_arcarc.py",
         "tests/test_hostcheck_property.py", "tests/test_hostcheck_shared.py",
         "tests/test_candidates.py"]


def test_host_build_is_clean_under_asan_and_ubsan(tmp_path):
    lib = build.build_hostcheck_sanitized(str(tmp_path / "libsphint_hostcheck_asan.so"))
    env = dict(os.environ)
    env.update(LD_PRELOAD=build.asan_runtime(), SPHINT_HOSTCHECK_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *FILES], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out and "failed" not in out, out[-2000:]
