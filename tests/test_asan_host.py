"""The host side of the library under AddressSanitizer, on the CPU: the CPU ABI tests
(argument validation before any device work; the multiplet, channel and transition-amplitude
helpers; the continued-fraction checks; the exported symbols) run again against a build whose
host code is instrumented (paper_1601_07728_amd/build.py, build(asan=True)), with the
sanitizer runtime preloaded.  An invalid host memory access aborts that run."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_abi_cpu_tests_pass_under_asan():
    rt = _runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm installation")
    from paper_1601_07728_amd import build as b
    srcs = [os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC)]
    if not os.path.exists(b.LIB_ASAN) or max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(b.LIB_ASAN):
        b.build(asan=True)
    # the host code is instrumented: it calls the sanitizer's access checks
    syms = subprocess.run(["nm", "-D", "--undefined-only", b.LIB_ASAN], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", OCEAN_BSE_LIB=b.LIB_ASAN)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr
    assert " passed" in r.stdout
