"""Host-side sanitizer runs (no GPU): the C oracle and the library's host
code built with AddressSanitizer + UndefinedBehaviorSanitizer (device code
unchanged), each exercised by its own CPU test suite in a subprocess that
preloads the sanitizer runtime.  Any report aborts that subprocess."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"       # the interpreter's own allocations outlive it
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    import oracle
    lib = oracle.build(out=str(tmp_path / "liblnbnn_oracle_san.so"), sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    out = _run({"LNBNN_ORACLE_LIB": lib, "LD_PRELOAD": asan},
               ["tests/test_oracle.py", "tests/test_oracle_fp8.py"])
    assert " passed" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1112_0059_amd import build
    if not os.path.exists(build.BUILD):
        pytest.skip("the regular build's objects are not there (run build() first)")
    lib = build.build_sanitized(str(tmp_path / "asan"))
    out = _run({"LNBNN_LIBRARY": lib, "LD_PRELOAD": build.asan_runtime()}, ["tests/test_abi.py"])
    assert " passed" in out
