"""Pins of the oracle's training-data functions beyond the one-step triple
(section 3.4, eq. 3.8-3.9): k flexible-GMRES steps and the augmentation by
linear combinations."""
import numpy as np
import pytest

from oracle import helm_oracle, unet_oracle as U
from paper_2203_11025_amd import inputs


def _setup(n=32, levels=2, seed=3):
    kap = inputs.smooth_medium(n, 3.0, seed=seed)
    gam = inputs.sponge_gamma(n, width=6)
    om = inputs.omega_for_ppw(n)
    H = helm_oracle.Hierarchy(kap, gam, om, levels)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return kap, gam, om, H, x


def test_one_step_equals_the_closed_form_minimiser():
    """k = 1 through the FGMRES iteration equals the closed-form one-step
    triple (alpha z with alpha minimising ||b - alpha A z||)."""
    _, _, _, H, x = _setup()
    r1, e1, its = U.training_triple_k(H, x, 1)
    r0, e0 = U.training_triple(H, x)
    assert its == 1
    assert np.linalg.norm(r1 - r0) <= 1e-12 * np.linalg.norm(r0)
    assert np.linalg.norm(e1 - e0) <= 1e-12 * np.linalg.norm(e0)


def test_k_steps_residual_is_consistent_and_nonincreasing():
    """A e = r to rounding for every k; since the SL V-cycle is a fixed
    linear preconditioner, k FGMRES steps minimise ||b - A x~|| over a
    growing space: ||r|| never increases with k."""
    kap, gam, om, H, x = _setup()
    prev = np.inf
    for k in (1, 2, 3, 5, 10):
        r, e, its = U.training_triple_k(H, x, k)
        assert its == k
        Ae = helm_oracle.apply(kap, gam, om, e)
        assert np.linalg.norm(Ae - r) <= 1e-10 * np.linalg.norm(r)
        nr = np.linalg.norm(r)
        assert nr <= prev * (1 + 1e-12)
        prev = nr


def test_k_steps_with_an_exact_preconditioner_solve_in_one_step():
    """On a one-level hierarchy the V-cycle is M^-1 with M the shifted
    operator; with beta = 0 it is A^-1 and one step already gives x~ = x."""
    n = 8
    kap = inputs.smooth_medium(n, 1.5, seed=1)
    gam = inputs.sponge_gamma(n, width=2)
    om = inputs.omega_for_ppw(n)
    H = helm_oracle.Hierarchy(kap, gam, om, 1, beta=0.0)
    x = np.random.default_rng(2).standard_normal((n, n)) + 0j
    r, e, its = U.training_triple_k(H, x, 3)
    assert np.linalg.norm(e) <= 1e-9 * np.linalg.norm(x)


def test_mix_keeps_the_triple_relation_and_is_the_matrix_product():
    kap, gam, om, H, x = _setup()
    rng = np.random.default_rng(9)
    rs, es = [], []
    for k in range(4):
        r, e = U.training_triple(H, x * (k + 1) + rng.standard_normal(x.shape))
        rs.append(r)
        es.append(e)
    c = rng.standard_normal((3, 4))
    r2, e2 = U.mix_triples(rs, es, c)
    for b in range(3):
        Ae = helm_oracle.apply(kap, gam, om, e2[b])
        assert np.linalg.norm(Ae - r2[b]) <= 1e-10 * np.linalg.norm(r2[b])
        ref = sum(c[b, j] * rs[j] for j in range(4))
        assert np.abs(r2[b] - ref).max() <= 1e-12 * np.abs(ref).max()
