"""Seeded synthetic inputs for the heterogeneous Helmholtz problem.

This module holds only input generation: slowness media, the absorbing-layer
attenuation field, the frequency rule, right-hand sides and random draws.  It
contains none of the solver's arithmetic, so that both the CPU oracle and the
GPU library can be fed from it without sharing any method code.

Problem definition followed here (paper section 2.1, eq. 2.1-2.3): the unit
square with an n x n array of unknowns, mesh width h = 1/n, slowness kappa(x)
and an attenuation field gamma(x) that carries the absorbing layer.  The
10-points-per-wavelength rule omega*kappa*h <= 2*pi/10 fixes omega.

All slowness and attenuation fields are returned as float32, the precision the
library accepts; the oracle promotes exactly these float32 values to float64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "omega_for_ppw",
    "sponge_gamma",
    "smooth_medium",
    "layered_medium",
    "constant_medium",
    "point_source",
    "source_positions",
    "point_sources",
    "complex_gaussian",
    "config_problem",
    "config_problems",
]


def omega_for_ppw(n: int, ppw: float = 10.0, kappa_max: float = 1.0) -> float:
    """Angular frequency with exactly `ppw` points per shortest wavelength.

    Section 2.1 states the rule omega * kappa * h <= 2*pi/10 for h = 1/n; this
    returns the equality case, omega = 2*pi*n / (ppw * kappa_max).
    """
    h = 1.0 / n
    return 2.0 * math.pi / (ppw * h * kappa_max)


def sponge_gamma(n: int, width: int = 16, interior: float = 0.01,
                 edge: float = 1.0) -> np.ndarray:
    """Attenuation field gamma(i, j) with a quadratic absorbing layer.

    The paper models the absorbing boundary layer through the attenuation
    gamma inside the mass term (section 2.1 and section 4); it gives neither
    the profile nor the edge value, so this uses a quadratic ramp:
    d(i) = min(i, n-1-i), s(d) = ((width - d)/width)^2 for d < width else 0,
    gamma = interior + (edge - interior) * max(s(d(i)), s(d(j))).
    """
    i = np.arange(n)
    d = np.minimum(i, n - 1 - i).astype(np.float64)
    s = np.where(d < width, ((width - d) / width) ** 2, 0.0)
    ramp = np.maximum(s[:, None], s[None, :])
    g = interior + (edge - interior) * ramp
    return g.astype(np.float32)


def _gaussian_filter_reflect(a: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    return gaussian_filter(a, sigma=sigma, mode="reflect", truncate=4.0)


def smooth_medium(n: int, sigma: float, seed: int, lo: float = 0.25,
                  hi: float = 1.0) -> np.ndarray:
    """Smooth random slowness: Gaussian-filtered white noise, mapped to [lo, hi].

    Stand-in for the paper's smoothed, normalised natural-image media
    (section 3.4.1): same grid size, value range and smoothing style, from
    seeded white noise instead of images.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    s = _gaussian_filter_reflect(w, sigma)
    s = (s - s.min()) / (s.max() - s.min())
    return (lo + (hi - lo) * s).astype(np.float32)


def layered_medium(n: int, seed: int, lo: float = 0.25, hi: float = 1.0,
                   perturb: float = 0.10) -> np.ndarray:
    """Layered slowness with 3-8 horizontal layers plus a smooth perturbation.

    Layer slownesses decrease with depth (velocity grows deeper, the usual
    geophysical setting mentioned in section 3.4.1); a smoothed-noise field
    scaled to [-1, 1] perturbs it multiplicatively by +-`perturb`.
    """
    rng = np.random.default_rng(seed)
    nlayers = int(rng.integers(3, 9))
    cuts = np.sort(rng.integers(1, n, size=nlayers - 1))
    vals = np.sort(rng.uniform(lo, hi, size=nlayers))[::-1]
    rows = np.zeros(n)
    start = 0
    for k, c in enumerate(list(cuts) + [n]):
        rows[start:c] = vals[k]
        start = c
    base = np.repeat(rows[:, None], n, axis=1)
    noise = _gaussian_filter_reflect(rng.standard_normal((n, n)), n / 32.0)
    noise = 2.0 * (noise - noise.min()) / (noise.max() - noise.min()) - 1.0
    out = np.clip(base * (1.0 + perturb * noise), lo, hi)
    return out.astype(np.float32)


def constant_medium(n: int, value: float = 1.0) -> np.ndarray:
    return np.full((n, n), value, dtype=np.float32)


def point_source(n: int, pos: tuple[int, int] | None = None) -> np.ndarray:
    """Right-hand side f = 1/h^2 at one grid point (the centre by default)."""
    if pos is None:
        pos = (n // 2, n // 2)
    f = np.zeros((n, n), dtype=np.complex64)
    f[pos] = float(n) * float(n)
    return f


def source_positions(n: int, count: int, seed: int, margin: int = 16) -> np.ndarray:
    """`count` seeded source positions, uniform in [margin, n-1-margin]^2."""
    rng = np.random.default_rng(seed)
    return rng.integers(margin, n - margin, size=(count, 2))


def point_sources(n: int, count: int, seed: int, margin: int = 16) -> np.ndarray:
    """Batch [count, n, n] of complex64 point-source right-hand sides."""
    pos = source_positions(n, count, seed, margin)
    b = np.zeros((count, n, n), dtype=np.complex64)
    for k, (i, j) in enumerate(pos):
        b[k, i, j] = float(n) * float(n)
    return b


def complex_gaussian(shape, seed: int) -> np.ndarray:
    """complex64 array with iid N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex64)


def config_problem(name: str) -> dict:
    """The named synthetic workloads (grid, medium, frequency, sources).

    plain128   : 128^2, kappa = 1, centre point source, 3 levels, FGMRES(10)
    plain512   : 512^2, smooth medium (sigma 16 cells, seed 1), 4 levels,
                 centre point source, FGMRES(20)
    multi1024  : 1024^2, smooth medium (sigma 32 cells, seed 2), 32 point
                 sources (seed 3), 5 levels, FGMRES(20)
    """
    sigma = None
    if name == "plain128":
        n = 128
        kappa = constant_medium(n)
        b = point_source(n)[None]
        levels, m = 3, 10
    elif name == "plain512":
        n = 512
        sigma = 16.0
        kappa = smooth_medium(n, sigma, seed=1)
        b = point_source(n)[None]
        levels, m = 4, 20
    elif name == "multi1024":
        n = 1024
        sigma = 32.0
        kappa = smooth_medium(n, sigma, seed=2)
        b = point_sources(n, 32, seed=3)
        levels, m = 5, 20
    else:
        raise ValueError(f"unknown workload {name!r}")
    return dict(n=n, kappa=kappa, gamma=sponge_gamma(n), omega=omega_for_ppw(n),
                b=b, levels=levels, m=m, tol=1e-7, sigma=sigma)


def config_problems(name: str, count: int | None = None) -> list:
    """The uneven batch: a list of problems (dicts as config_problem gives).

    uneven24 : 24 layered media (3-8 seeded horizontal layers, slowness in
               [0.25, 1] with a +/-10% smooth perturbation, seed 100 + k) of
               sizes drawn from {256, 512, 1024, 2048} (seed 4), 8 point
               sources each (seed 200 + k), omega for 10 points per
               wavelength, the levels rule of the other workloads (coarsest
               64^2), FGMRES(20) to 1e-7.  `count` keeps the first count media.
    uneven6  : six layered media, one of each size 256^2..2048^2 and two more
               (256^2, 512^2), 8 sources each, the same recipe.
    """
    if name == "uneven24":
        sizes = [int(v) for v in np.random.default_rng(4).choice([256, 512, 1024, 2048], size=24)]
    elif name == "uneven6":
        sizes = [256, 512, 1024, 2048, 256, 512]
    else:
        raise ValueError(f"unknown workload {name!r}")
    if count is not None:
        sizes = sizes[:count]
    out = []
    for k, n in enumerate(sizes):
        levels = 1
        while (n >> (levels - 1)) > 64:
            levels += 1
        out.append(dict(n=n, kappa=layered_medium(n, seed=100 + k), gamma=sponge_gamma(n),
                        omega=omega_for_ppw(n), b=point_sources(n, 8, seed=200 + k), levels=levels, m=20,
                        tol=1e-7, sigma=None))
    return out
