"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer: the library is
rebuilt with the host compilation sanitized (device code unchanged) and the CPU ABI tests
(exports, argument validation, refusals before any device work) run against it in a child
process with the sanitizer runtime preloaded.  Any report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _stale(lib, src_dirs):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    for d in src_dirs:
        for f in os.listdir(d):
            if f.endswith((".cpp", ".hip", ".h")) and os.path.getmtime(os.path.join(d, f)) > t:
                return True
    return False


def test_abi_host_code_under_sanitizers():
    from paper_2208_12335_amd import build_sanitize as bs
    if _stale(bs.LIB_SAN, [bs.CSRC, os.path.join(ROOT, "include")]):
        bs.build()
    env = dict(os.environ, LD_PRELOAD=bs.runtime(), AIMS_LIB=bs.LIB_SAN,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    print(p.stdout[-2000:])
    assert p.returncode == 0, p.stdout[-4000:]
    assert "ERROR: AddressSanitizer" not in p.stdout and "runtime error" not in p.stdout
