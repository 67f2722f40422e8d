"""Pins of the oracle's block FGMRES (section 4: block restarted FGMRES(10),
block size 10): block size 1 is the plain FGMRES oracle; with the identity
preconditioner the k-step iterate minimises the residual over the block
Krylov space (dense least squares); with the SL cycle it solves the system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import block_fgmres as BF, helm_oracle
from paper_2203_11025_amd import inputs


def _setup(n=32, levels=2, seed=2):
    kap = inputs.smooth_medium(n, 3.0, seed=seed)
    gam = inputs.sponge_gamma(n, width=6)
    om = inputs.omega_for_ppw(n)
    return kap, gam, om, helm_oracle.Hierarchy(kap, gam, om, levels)


def test_block_size_one_is_fgmres():
    kap, gam, om, H = _setup()
    b = inputs.point_source(32)
    x1, st1 = BF.block_fgmres(H, b[None], m=10, tol=1e-9)
    x0, st0 = H.fgmres(b, m=10, tol=1e-9)
    assert st1["iterations"] == st0["iterations"]
    assert np.linalg.norm(x1[0] - x0) <= 1e-10 * np.linalg.norm(x0)


@pytest.mark.parametrize("k,s", [(1, 3), (3, 2), (4, 3)])
def test_identity_preconditioner_minimises_over_the_block_krylov_space(k, s):
    n = 8
    kap, gam, om, H = _setup(n=n, levels=1)
    rng = np.random.default_rng(k * 10 + s)
    B = rng.standard_normal((s, n, n)) + 1j * rng.standard_normal((s, n, n))
    X, st = BF.block_fgmres(H, B, m=k, tol=0.0, maxit=k, prec=lambda v: v)
    assert st["iterations"] == k
    A = helm_oracle.operator_matrix(kap, gam, om).toarray()
    Bm = B.reshape(s, -1).T
    # span{B, AB, ..., A^(k-1) B}, kept orthonormal by dense QR at every
    # power (the monomial basis itself is too ill-conditioned to solve on)
    K = np.linalg.qr(Bm)[0]
    for _ in range(k - 1):
        K = np.linalg.qr(np.concatenate([K, A @ K[:, -s:]], axis=1))[0]
    C = np.linalg.lstsq(A @ K, Bm, rcond=None)[0]
    ref = (K @ C).T.reshape(s, n, n)
    assert np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)


def test_sl_preconditioned_block_solve_reaches_the_exact_solution():
    kap, gam, om, H = _setup()
    B = inputs.point_sources(32, 3, seed=4, margin=6).astype(complex)
    X, st = BF.block_fgmres(H, B, m=10, tol=1e-10)
    assert max(st["true_relres"]) <= 1e-10
    Am = helm_oracle.operator_matrix(kap, gam, om).tocsc()
    for k in range(3):
        ref = spl.spsolve(Am, B[k].ravel()).reshape(32, 32)
        assert np.linalg.norm(X[k] - ref) <= 1e-8 * np.linalg.norm(ref)
