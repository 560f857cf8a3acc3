"""The C ABI's argument checks under host AddressSanitizer and
UndefinedBehaviorSanitizer: the library's host code is built with both
(`python -m paper_2208_02734_amd.build --sanitize`, device code as usual)
and the CPU ABI tests run against it in a child process with the ASan
runtime preloaded; any report ends the child with an error.  CPU only."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2208_02734_amd")
ASAN_LIB = os.path.join(PKG, "_lib_asan", "libmask.so")


def _runtime():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


def _stale():
    if not os.path.exists(ASAN_LIB):
        return True
    built = os.path.getmtime(ASAN_LIB)
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + [os.path.join(ROOT, "include", "mask.h")]
    return any(os.path.getmtime(s) > built for s in srcs)


@pytest.mark.slow
def test_abi_argument_checks_under_asan_and_ubsan():
    rt = _runtime()
    if rt is None or shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
        pytest.skip("no hipcc or sanitizer runtime")
    if _stale():
        sys.path.insert(0, ROOT)
        from paper_2208_02734_amd import build as b
        b.build(jobs=min(8, os.cpu_count() or 1), sanitize=True)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "MASK_LIBRARY": ASAN_LIB,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    probe = ("import ctypes, paper_2208_02734_amd as pk; L = pk.lib(); "
             "assert pk.LIB_PATH.endswith('_lib_asan/libmask.so'), pk.LIB_PATH; "
             "ctypes.CDLL(None).__asan_init; print('sanitized library loaded')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0 and "sanitized library loaded" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
