"""The host code of the library (container header parser and writer, host
range coder, configuration checks, the C-ABI argument handling) under
AddressSanitizer and UndefinedBehaviorSanitizer: the library is rebuilt with
both sanitizers on its host code only (build.py --sanitize; the gfx950 code
object is unchanged) and the host ABI tests, including the mutated-header and
garbage-payload cases, run against it in a child process with the ASan
runtime preloaded.  Any report aborts the child and fails this test."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_under_asan_and_ubsan():
    from paper_2507_18969_amd import build as B
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    rt = B.asan_runtime()
    if not rt or not os.path.exists(rt):
        pytest.skip("compiler ASan runtime not found")
    lib = B.build(jobs=min(8, os.cpu_count() or 1), verbose=False, sanitize=True)
    env = dict(os.environ, EDPC_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out
