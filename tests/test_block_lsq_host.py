"""The block FGMRES least squares (host code of the library) on the CPU.

Block FGMRES (section 4) picks Y = argmin ||E_1 beta - Hbar Y||_F over the
block Hessenberg matrix Hbar of a cycle.  The library reduces Hbar one block
column at a time with Householder reflections (``csrc/block_lsq.h``); this
test builds that header alone with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and compares, after every block column, the
solution and the per-right-hand-side residual norms with numpy's dense least
squares on the leading columns.  CPU only.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2203_11025_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("lsq") / "block_lsq")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", CSRC, "-o", exe,
           os.path.join(HERE, "block_lsq_driver.cpp")]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0 and ("asan" in p.stderr or "ubsan" in p.stderr):
        pytest.skip("g++ sanitizer runtimes are not installed")
    assert p.returncode == 0, p.stderr
    return exe


def _hessenberg(rng, s, m):
    M1, MS = (m + 1) * s, m * s
    H = np.zeros((M1, MS), np.complex128)
    for j in range(m):
        rows = (j + 2) * s
        H[:rows, j * s:(j + 1) * s] = rng.standard_normal((rows, s)) + 1j * rng.standard_normal((rows, s))
        # sub-diagonal block upper triangular, as Cholesky QR leaves it
        H[(j + 1) * s:rows, j * s:(j + 1) * s] = np.triu(H[(j + 1) * s:rows, j * s:(j + 1) * s])
    beta = np.triu(rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s)))
    return beta, H


def _run(driver, tmp_path, s, m, beta, H):
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([s, m], np.int32).tofile(f)
        np.ascontiguousarray(beta, np.complex128).tofile(f)
        np.ascontiguousarray(H, np.complex128).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([driver, str(fin), str(fout)], capture_output=True, text=True, timeout=120, env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    raw = np.fromfile(fout, np.uint8)
    out, off = [], 0
    for j in range(m):
        res = raw[off:off + 8 * s].view(np.float64)
        off += 8 * s
        ny = (j + 1) * s * s
        Y = raw[off:off + 16 * ny].view(np.complex128).reshape((j + 1) * s, s)
        off += 16 * ny
        out.append((res, Y))
    assert off == raw.size
    return out


@pytest.mark.parametrize("s,m,seed", [(1, 10, 0), (3, 5, 1), (10, 10, 2), (16, 4, 3)])
def test_block_lsq_matches_dense_least_squares(driver, tmp_path, s, m, seed):
    rng = np.random.default_rng(seed)
    beta, H = _hessenberg(rng, s, m)
    out = _run(driver, tmp_path, s, m, beta, H)
    for j, (res, Y) in enumerate(out):
        rows, cols = (j + 2) * s, (j + 1) * s
        E = np.zeros((rows, s), np.complex128)
        E[:s] = beta
        Yref = np.linalg.lstsq(H[:rows, :cols], E, rcond=None)[0]
        rref = np.linalg.norm(E - H[:rows, :cols] @ Yref, axis=0)
        scale = np.linalg.norm(Yref) + 1.0
        assert np.abs(Y - Yref).max() <= 1e-10 * scale, (j, np.abs(Y - Yref).max())
        assert np.allclose(res, rref, rtol=1e-10, atol=1e-12 * np.linalg.norm(beta)), (j, res, rref)


def test_block_lsq_zero_column(driver, tmp_path):
    """A vanishing sub-diagonal block leaves the reflections of its columns
    unset; the reduction still returns the least-squares solution of the
    columns before it and a zero residual there."""
    s, m = 2, 3
    rng = np.random.default_rng(7)
    beta, H = _hessenberg(rng, s, m)
    H[:, s:2 * s] = 0.0
    out = _run(driver, tmp_path, s, m, beta, H)
    res0, Y0 = out[0]
    E = np.zeros((2 * s, s), np.complex128)
    E[:s] = beta
    Yref = np.linalg.lstsq(H[:2 * s, :s], E, rcond=None)[0]
    assert np.abs(Y0 - Yref).max() <= 1e-10 * (np.linalg.norm(Yref) + 1)
    res1, Y1 = out[1]
    assert np.all(np.isfinite(Y1)) and np.all(Y1[s:2 * s] == 0.0)
    assert np.allclose(res1, res0, rtol=1e-12)
