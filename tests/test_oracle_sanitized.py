"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a host
driver (oracle/sanitize_driver.cpp) runs every exported entry point (sweeps,
corrected and full-symbol iterations, transforms, tables, marches with each
corrector and trial rule, the discrete adjoint, the cavity pieces) on tiny 2D
and 3D grids in a build with both sanitizers and recovery off, so any
out-of-bounds or misaligned access, use after free or undefined arithmetic
ends the run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_san")
    src = os.path.join(ROOT, "oracle", "sanitize_driver.cpp")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.run(["g++"] + flags + [src, "-o", exe], check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the run environment may preload a library of
    # its own ahead of the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle run: ok" in r.stdout
    assert "runtime error" not in r.stderr
