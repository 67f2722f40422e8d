"""Independent constructions used to pin the oracle.

These build the paper's operators a second way, from one-dimensional
matrices and Kronecker products with scipy, instead of the oracle's stencil
loops.  They are themselves pinned by the closed-form DST-I eigenpairs of the
constant-coefficient operator (tests/test_oracle_pins.py).
"""
import numpy as np
import scipy.sparse as sp


def second_difference(n):
    """1D matrix tridiag(-1, 2, -1) (zero Dirichlet ghosts)."""
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1],
                    shape=(n, n), format="csr")


def helmholtz_matrix(kappa, gamma, omega, shift=0.0, h=None):
    """Sparse operator (L1 (x) I + I (x) L1)/h^2 - diag(omega^2 kappa^2 (1 - i(gamma+shift)))."""
    kappa = np.asarray(kappa, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    n = kappa.shape[0]
    h = 1.0 / n if h is None else h
    T = second_difference(n)
    Id = sp.identity(n, format="csr")
    lap = (sp.kron(T, Id) + sp.kron(Id, T)) / (h * h)
    mass = omega ** 2 * kappa.ravel() ** 2 * (1 - 1j * (gamma.ravel() + shift))
    return (lap - sp.diags(mass)).tocsc()


def prolong_1d(nc):
    """1D linear interpolation n = 2 nc fine points from nc coarse points.

    Coarse point I sits at fine 2I; fine 2I+1 lies halfway to coarse I+1
    (which is the zero ghost for I = nc - 1)."""
    n = 2 * nc
    P = np.zeros((n, nc))
    for I in range(nc):
        P[2 * I, I] = 1.0
        if 2 * I + 1 < n:
            P[2 * I + 1, I] = 0.5
        if 2 * I - 1 >= 0:
            P[2 * I - 1, I] = 0.5
    return P


def restrict_1d(nc):
    """1D full weighting (1/4, 1/2, 1/4) centred on fine 2I."""
    n = 2 * nc
    R = np.zeros((nc, n))
    for I in range(nc):
        for a, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            if 0 <= 2 * I + a < n:
                R[I, 2 * I + a] = w
    return R


def dst_mode(n, k, l):
    i = np.arange(1, n + 1)
    return np.outer(np.sin(np.pi * k * i / (n + 1)), np.sin(np.pi * l * i / (n + 1)))


def dst_eigenvalue(n, k, l, kappa, gamma, omega, shift=0.0):
    """Eigenvalue of the constant-coefficient operator on the DST-I mode (k, l)."""
    h = 1.0 / n
    lap = (4 - 2 * np.cos(np.pi * k / (n + 1)) - 2 * np.cos(np.pi * l / (n + 1))) / h ** 2
    return lap - omega ** 2 * kappa ** 2 * (1 - 1j * (gamma + shift))
