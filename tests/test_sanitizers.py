"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU needed): both are rebuilt with the sanitizers
(the library's device code unchanged), and the host and oracle test modules run in a
child process that preloads the sanitizer runtime and loads those builds; any report
ends it with an error."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HOST_TESTS = ["test_host.py", "test_oracle_sum.py", "test_oracle_tables.py",
              "test_oracle_model.py", "test_oracle_resolution.py"]


def _asan_runtime():
    found = sorted(glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    return found[-1] if found else None


def test_host_code_and_oracle_under_asan_ubsan():
    rt = _asan_runtime()
    if rt is None or not os.path.exists(os.path.join(ROCM, "bin", "hipcc")):
        pytest.skip("clang sanitizer runtime or hipcc not available")
    sys.path.insert(0, os.path.join(ROOT, "paper_1301_3968_amd"))
    try:
        import build as libbuild
    finally:
        sys.path.pop(0)
    import oracle
    lib = libbuild.build(sanitize=True)
    olib = oracle.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, DEDISP_LIB=lib, ORACLE_LIB=olib,
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:"
                            "halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child loads the sanitized builds (checked in its memory map) ...
    probe = ("import paper_1301_3968_amd, oracle; oracle.lib(); "
             "m = open('/proc/self/maps').read(); "
             "assert 'libdedisp_san.so' in m and 'liboracle_san.so' in m, 'not loaded'")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    # ... and runs the host and oracle tests with them
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p",
                        "no:cacheprovider"] + [os.path.join("tests", t) for t in HOST_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
