"""The oracle (plain C) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on small lattices (cubic, stars of 2, 21
and 40 struts, a capsule with an isolated node) through
oracle/sanitize_main.c, which reads every output array: no sanitizer
report, every lattice meshed with valid triangle indices."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-pthread", os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_main.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert out.count("triangles") == 5 and "BAD INDEX" not in out, out
