"""Pins of the oracle's GMRES coarsest-level solver (section 4's setting:
GMRES(10) with the Jacobi diagonal preconditioner on the coarsest grid of
the SL V-cycle, then Algorithm 1's post-relaxation), against dense linear
algebra written independently here."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import helm_oracle
from paper_2203_11025_amd import inputs


def _medium(n, seed):
    kap = inputs.smooth_medium(n, 2.0, seed=seed)
    gam = inputs.sponge_gamma(n, width=max(1, n // 8))
    return kap, gam, inputs.omega_for_ppw(n)


def _jacobi(Mm, f, x, w=0.8):
    d = Mm.diagonal()
    return x + w * (f - Mm @ x) / d


def test_full_krylov_space_is_an_exact_solve():
    """k = number of unknowns: the Krylov space is the whole space, the
    coarse solve is M^-1 f, and the post-relaxation leaves it unchanged."""
    n = 4
    kap, gam, om = _medium(n, 1)
    H = helm_oracle.Hierarchy(kap, gam, om, 1, coarse_gmres=n * n)
    f = np.random.default_rng(0).standard_normal((n, n)) + 1j * np.random.default_rng(1).standard_normal((n, n))
    Mm = helm_oracle.operator_matrix(kap, gam, om, shift=0.5)
    ref = spl.spsolve(Mm.tocsc(), f.ravel()).reshape(n, n)
    v = H.vcycle(f)
    assert np.linalg.norm(v - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", [1, 3, 10])
def test_k_steps_minimise_the_residual_over_the_preconditioned_krylov_space(k):
    """x = argmin ||f - M x|| over x in D^-1 span{(M D^-1)^i f, i < k}, by a
    dense least-squares solve over the explicit (orthonormalised) Krylov
    vectors, then one damped Jacobi sweep (weight 0.8) on M."""
    n = 8
    kap, gam, om = _medium(n, 2)
    H = helm_oracle.Hierarchy(kap, gam, om, 1, coarse_gmres=k)
    rng = np.random.default_rng(k)
    f = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Mm = helm_oracle.operator_matrix(kap, gam, om, shift=0.5).toarray()
    dinv = 1.0 / np.diag(Mm)
    K = np.empty((n * n, k), dtype=complex)
    v = f.ravel().copy()
    for i in range(k):
        K[:, i] = v
        v = Mm @ (dinv * v)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(Mm @ (dinv[:, None] * Q), f.ravel(), rcond=None)
    x = dinv * (Q @ y)
    ref = _jacobi(Mm, f.ravel(), x).reshape(n, n)
    got = H.vcycle(f)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_three_level_cycle_with_gmres_coarsest_is_homogeneous_and_close_to_exact():
    """The cycle is positively (indeed complex-) homogeneous; with many
    coarse steps it approaches the exact-coarsest cycle."""
    n = 32
    kap, gam, om = _medium(n, 3)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H10 = helm_oracle.Hierarchy(kap, gam, om, 3, coarse_gmres=10)
    a = H10.vcycle(f)
    c = 2.5 - 1.5j
    assert np.linalg.norm(H10.vcycle(c * f) - c * a) <= 1e-12 * np.linalg.norm(c * a)
    He = helm_oracle.Hierarchy(kap, gam, om, 3)
    H64 = helm_oracle.Hierarchy(kap, gam, om, 3, coarse_gmres=64)
    ve, v64 = He.vcycle(f), H64.vcycle(f)
    assert np.linalg.norm(v64 - ve) <= 1e-6 * np.linalg.norm(ve)
    assert np.linalg.norm(a - ve) > np.linalg.norm(v64 - ve)
