"""The library's host-side logic under AddressSanitizer (CPU): the host tests (order selection against the
oracle, functionals' host parts, symbol and argument checks) run in a child process that loads the
host-sanitizer build of the library (paper_1806_11456_amd/libpmg_asan_host.so, built by build()) with the
sanitizer runtime preloaded; any heap or stack error in the host code aborts that process."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "paper_1806_11456_amd", "libpmg_asan_host.so")


def _runtime():
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


@pytest.mark.skipif(not os.path.exists(ASAN_LIB), reason="host-sanitizer library not built (build() builds it)")
@pytest.mark.skipif(_runtime() is None, reason="no AddressSanitizer runtime in the ROCm toolchain")
def test_host_logic_under_address_sanitizer():
    with open(ASAN_LIB, "rb") as f:
        assert b"__asan_report_load8" in f.read(), "the library is not instrumented"
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _runtime() + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["PMG_LIB"] = ASAN_LIB
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_adapt_host.py", "test_functionals_host.py", "test_abi.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "AddressSanitizer" not in r.stderr
