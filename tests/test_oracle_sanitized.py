"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds ``oracle_sanitize_driver.c`` (which includes ``oracle/helm_oracle.c``)
with gcc's ASan + UBSan, aborting on the first finding, and runs every entry
point of the oracle on small grids: the stencil of eq. 2.2, the transfers of
eq. 2.9 (checked adjoint, P = 4 R^T), the banded direct solve, V-cycles with
an exact and a GMRES-solved coarsest level (Algorithm 1, section 4) and
FGMRES, plus its argument checks.  CPU only.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _build(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0 and ("asan" in p.stderr or "ubsan" in p.stderr):
        pytest.skip("gcc sanitizer runtimes are not installed: " + p.stderr.strip()[:200])
    assert p.returncode == 0, p.stderr
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert p.stdout.strip().endswith("OK"), p.stdout
