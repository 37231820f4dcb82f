"""The runtime's host code under AddressSanitizer and UndefinedBehaviorSanitizer: the library is built
with host-side instrumentation (device code as usual; paper_2601_16949_amd/build.py --sanitize) and the
CPU-side ABI tests run against it in a child process with the sanitizer runtime preloaded, stopping at
the first report.  No GPU is needed: these tests exercise the layout arithmetic, the argument checks
and the error paths that run before any device work."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2601_16949_amd import build as B  # noqa: E402


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _sanitized_library():
    srcs = B.sources()
    if os.path.exists(B.SAN_OUT) and os.path.getmtime(B.SAN_OUT) >= max(os.path.getmtime(f) for f in srcs):
        return B.SAN_OUT
    return B.build(jobs=min(8, os.cpu_count() or 1), verbose=False, sanitize=True)


@pytest.fixture(scope="module")
def san_env():
    rt = _asan_runtime()
    if rt is None or not os.path.exists(B.HIPCC):
        pytest.skip("clang sanitizer runtime or hipcc not available")
    lib = _sanitized_library()
    env = dict(os.environ, RTTDA_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return lib, env


def test_library_is_instrumented(san_env):
    lib, env = san_env
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    maps = subprocess.run([sys.executable, "-c", "print(open('/proc/self/maps').read())"], env=env,
                          capture_output=True, text=True).stdout
    assert "libclang_rt.asan" in maps


def test_abi_tests_clean_under_sanitizers(san_env):
    lib, env = san_env
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "passed" in out and "ERROR: AddressSanitizer" not in out \
        and "runtime error" not in out, out[-4000:]
