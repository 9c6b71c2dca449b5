"""The C ABI's host code under AddressSanitizer: the validation, workspace
and plan bookkeeping tests of test_abi.py run against libttgfx_asan.so (the
same sources with the host pass instrumented; build.py --asan) with the ASan
runtime preloaded.  No device work: any out-of-bounds or use-after-free in
descriptor checks, arena sizing or policy code fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    sys.path.insert(0, ROOT)
    from paper_1801_01928_amd.build import ASAN_LIB, asan_runtime
    return ASAN_LIB, asan_runtime()


def test_abi_under_host_asan():
    lib, rt = _runtime()
    if not os.path.exists(lib):
        pytest.skip("libttgfx_asan.so not built (python paper_1801_01928_amd/build.py --asan)")
    if not rt:
        pytest.skip("no AddressSanitizer runtime next to the ROCm clang")
    env = dict(os.environ, LD_PRELOAD=rt, TTGFX_LIB=lib, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    # the instrumented library is the one the binding loads
    probe = ("import sys; sys.path.insert(0, %r); import paper_1801_01928_amd as tt; tt.load(); "
             "maps = open('/proc/self/maps').read(); assert 'libttgfx_asan.so' in maps; "
             "assert 'libttgfx.so' not in maps.replace('libttgfx_asan.so', ''); print('asan library loaded')" % ROOT)
    p = subprocess.run([sys.executable, "-c", probe], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=300)
    assert p.returncode == 0 and "asan library loaded" in p.stdout, p.stdout[-3000:]
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=600)
    assert "AddressSanitizer" not in p.stdout, p.stdout[-5000:]
    assert p.returncode == 0, p.stdout[-5000:]
