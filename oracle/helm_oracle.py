"""ctypes wrapper of the C oracle (``helm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the plain FP64 CPU reference the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library.

Fields are numpy arrays of shape (n, n), row-major, complex128 for grid
functions and float64 for coefficients (callers pass the float32 inputs; they
are promoted exactly).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "helm_oracle.c")
_LIB = os.path.join(_HERE, "libhelm_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_dp = C.POINTER(C.c_double)


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int),
                ("converged", C.c_int), ("true_relres", C.c_double)]


PREC_FN = C.CFUNCTYPE(None, C.c_void_p, _dp, _dp)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.orc_apply.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_residual.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, C.c_double,
                                   _dp, _dp, _dp]
        L.orc_jacobi.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, C.c_double,
                                 C.c_double, _dp, _dp]
        L.orc_restrict.argtypes = [C.c_int, _dp, _dp]
        L.orc_prolong_add.argtypes = [C.c_int, _dp, _dp]
        L.orc_inject.argtypes = [C.c_int, _dp, _dp]
        L.orc_band_solve.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, C.c_double, _dp]
        L.orc_band_solve.restype = C.c_int
        L.orc_hier_create.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, C.c_double,
                                      C.c_double]
        L.orc_hier_create.restype = C.c_void_p
        L.orc_hier_free.argtypes = [C.c_void_p]
        L.orc_hier_level_n.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_level_n.restype = C.c_int
        L.orc_hier_level_kappa.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_level_kappa.restype = _dp
        L.orc_hier_level_gamma.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_level_gamma.restype = _dp
        L.orc_vcycle.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_vcycle.restype = C.c_int
        L.orc_fgmres.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                 C.c_int, _dp, _dp, _dp, C.POINTER(_Stats)]
        L.orc_fgmres.restype = C.c_int
        L.orc_hier_residual_A.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_hier_set_coarse_gmres.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_set_coarse_gmres.restype = C.c_int
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _r(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp)


def apply(kappa, gamma, omega, x, shift=0.0, h=None):
    """y = Op x on one grid (eq. 2.1-2.2); shift = beta gives the SL operator."""
    k, g, xx = _r(kappa), _r(gamma), _c(x)
    n = k.shape[0]
    h = 1.0 / n if h is None else h
    y = np.empty_like(xx)
    lib().orc_apply(n, h, omega, _p(k), _p(g), shift, _p(xx), _p(y))
    return y


def residual(kappa, gamma, omega, f, x, shift=0.0, h=None):
    k, g, ff, xx = _r(kappa), _r(gamma), _c(f), _c(x)
    n = k.shape[0]
    h = 1.0 / n if h is None else h
    r = np.empty_like(xx)
    lib().orc_residual(n, h, omega, _p(k), _p(g), shift, _p(ff), _p(xx), _p(r))
    return r


def jacobi(kappa, gamma, omega, f, x, shift=0.0, weight=0.8, h=None):
    """One damped Jacobi sweep; returns the updated copy of x."""
    k, g, ff = _r(kappa), _r(gamma), _c(f)
    xx = _c(x).copy()
    n = k.shape[0]
    h = 1.0 / n if h is None else h
    lib().orc_jacobi(n, h, omega, _p(k), _p(g), shift, weight, _p(ff), _p(xx))
    return xx


def restrict(f):
    ff = _c(f)
    n = ff.shape[0]
    fc = np.empty((n // 2, n // 2), dtype=np.complex128)
    lib().orc_restrict(n, _p(ff), _p(fc))
    return fc


def prolong(ec, n=None):
    """P ec on the fine grid (fine size 2 * coarse size)."""
    e = _c(ec)
    n = 2 * e.shape[0] if n is None else n
    out = np.zeros((n, n), dtype=np.complex128)
    lib().orc_prolong_add(n, _p(e), _p(out))
    return out


def inject(field):
    f = _r(field)
    n = f.shape[0]
    c = np.empty((n // 2, n // 2), dtype=np.float64)
    lib().orc_inject(n, _p(f), _p(c))
    return c


def band_solve(kappa, gamma, omega, b, shift=0.0, h=None):
    """Direct solve Op x = b by banded LU with partial pivoting."""
    k, g = _r(kappa), _r(gamma)
    x = _c(b).copy()
    n = k.shape[0]
    h = 1.0 / n if h is None else h
    rc = lib().orc_band_solve(n, h, omega, _p(k), _p(g), shift, _p(x))
    if rc != 0:
        raise ArithmeticError("singular pivot in banded LU")
    return x


class Hierarchy:
    """SL multigrid hierarchy (section 2.2) plus the FGMRES driver."""

    def __init__(self, kappa, gamma, omega, levels, beta=0.5, weight=0.8, coarse_gmres=0):
        """coarse_gmres = k > 0: the coarsest level is solved by k GMRES
        steps with the Jacobi preconditioner from zero, then one damped
        Jacobi post-relaxation (section 4's setting); 0: exactly."""
        self.kappa0 = _r(kappa)
        self.gamma0 = _r(gamma)
        self.n = self.kappa0.shape[0]
        self.omega = float(omega)
        self.levels = levels
        self.beta = beta
        self.weight = weight
        h = lib().orc_hier_create(self.n, levels, self.omega, _p(self.kappa0),
                                  _p(self.gamma0), beta, weight)
        if not h:
            raise ValueError("invalid hierarchy (size / levels) or singular coarse operator")
        self._h = h
        self.coarse_gmres = int(coarse_gmres)
        if lib().orc_hier_set_coarse_gmres(h, self.coarse_gmres) != 0:
            raise ValueError("coarse_gmres must be >= 0")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_hier_free(self._h)
            self._h = None

    def level(self, l):
        n = lib().orc_hier_level_n(self._h, l)
        k = np.ctypeslib.as_array(lib().orc_hier_level_kappa(self._h, l), shape=(n, n)).copy()
        g = np.ctypeslib.as_array(lib().orc_hier_level_gamma(self._h, l), shape=(n, n)).copy()
        return n, k, g

    def vcycle(self, f):
        ff = _c(f)
        v = np.empty_like(ff)
        lib().orc_vcycle(self._h, _p(ff), _p(v))
        return v

    def residual_A(self, f, x):
        ff, xx = _c(f), _c(x)
        r = np.empty_like(ff)
        lib().orc_hier_residual_A(self._h, _p(ff), _p(xx), _p(r))
        return r

    def fgmres(self, b, m=10, tol=1e-7, maxit=20000, prec=None, history=False):
        """Solve A x = b.  prec: None (SL V-cycle) or a python callable v -> z.

        Returns (x, stats dict) and, with history=True, the implicit residual
        history ||r_k|| / ||b||.
        """
        bb = _c(b)
        x = np.empty_like(bb)
        hist = np.zeros(maxit + 1)
        st = _Stats()
        cb = None
        if prec is not None:
            n = self.n

            def _cb(_ctx, pin, pout):
                vin = np.ctypeslib.as_array(pin, shape=(n * n * 2,)).view(np.complex128)
                z = _c(prec(vin.reshape(n, n).copy()))
                vout = np.ctypeslib.as_array(pout, shape=(n * n * 2,)).view(np.complex128)
                vout[:] = z.ravel()

            cb = PREC_FN(_cb)
        lib().orc_fgmres(self._h, C.cast(cb, C.c_void_p) if cb else None, None, m, tol,
                         maxit, _p(bb), _p(x), _p(hist), C.byref(st))
        stats = dict(iterations=st.iterations, restarts=st.restarts,
                     converged=bool(st.converged), true_relres=st.true_relres)
        if history:
            return x, stats, hist[: st.iterations + 1]
        return x, stats


def convergence_factor(hist, reduction=1e6):
    """Eq. 4.1: rho = (||r_T|| / ||r_0||)^(1/T), T = first iteration reaching
    the given reduction (or the last iteration if it is never reached)."""
    hist = np.asarray(hist)
    hit = np.nonzero(hist <= hist[0] / reduction)[0]
    T = int(hit[0]) if hit.size else len(hist) - 1
    if T == 0:
        return 0.0, 0
    return float((hist[T] / hist[0]) ** (1.0 / T)), T


def operator_matrix(kappa, gamma, omega, shift=0.0, h=None):
    """The operator of eq. 2.2 (shift = beta: the SL operator of eq. 2.4) as a
    scipy sparse matrix on the n x n unknowns (row-major, zero outside):
    diagonal 4/h^2 - omega^2 kappa^2 (1 - i (gamma + shift)), -1/h^2 for each
    of the four neighbours inside the grid."""
    import scipy.sparse as sp

    k, g = _r(kappa), _r(gamma)
    n = k.shape[0]
    h = 1.0 / n if h is None else h
    ih2 = 1.0 / (h * h)
    idx = np.arange(n * n).reshape(n, n)
    diag = 4.0 * ih2 - omega ** 2 * k.ravel() ** 2 * (1 - 1j * (g.ravel() + shift))
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag]
    for a, b in (((slice(1, None), slice(None)), (slice(None, -1), slice(None))),
                 ((slice(None, -1), slice(None)), (slice(1, None), slice(None))),
                 ((slice(None), slice(1, None)), (slice(None), slice(None, -1))),
                 ((slice(None), slice(None, -1)), (slice(None), slice(1, None)))):
        r, c = idx[a].ravel(), idx[b].ravel()
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.size, -ih2, dtype=complex))
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, n * n))


def direct_solver(kappa, gamma, omega, shift=0.0):
    """x = Op^-1 b by a sparse LU factorisation (SuperLU, factored once) of
    operator_matrix: the exact solution of the discrete system, for reference
    solutions at sizes where the plain-C FGMRES is slow.  Returns b -> x."""
    import scipy.sparse.linalg as spl

    n = _r(kappa).shape[0]
    lu = spl.splu(operator_matrix(kappa, gamma, omega, shift), permc_spec="COLAMD")
    return lambda b: lu.solve(_c(b).ravel()).reshape(n, n)
