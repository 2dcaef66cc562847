"""Seeded synthetic inputs for the Gaussian-process likelihood path.

This module only draws numbers: point sets on the unit square, prediction
points, standard-normal vectors and a smooth random field for the response.
It evaluates no covariance function, factors nothing and solves nothing, so
both the GPU path and the CPU reference can take their inputs from here
without sharing any of the method's arithmetic.

Recipes (all numpy PCG64 through ``numpy.random.default_rng(seed)``):

* ``uniform_points(n, seed)``: n points i.i.d. uniform on [0, 1]^2.
* ``mixture_points(n, seed)``: a 50-component Gaussian mixture on [0, 1]^2,
  centres uniform on the square, equal weights, isotropic sd 0.02; points
  that fall outside the square are redrawn.
* ``normals(n, seed)``: i.i.d. N(0, 1) draws (used as z in y = L z).
* ``smooth_field(X, seed, ...)``: a sum of random cosines
  sqrt(2 s2 / K) * sum_k cos(w_k . x + b_k) with w_k ~ N(0, I / ell^2) and
  b_k ~ U[0, 2 pi), plus i.i.d. N(0, t2) noise. It has the length scale and
  amplitude of the workloads' fields; it is a stand-in response for sizes at
  which a dense factor of the model covariance is too slow to draw y from.
* ``batch_sizes(nb, seed, lo, hi)``: problem sizes uniform on {lo..hi}.
* ``spectral_points(n_phase, n_wave, seed)``: (phase, log-wavelength, noise
  variance) rows on the grid layout of the paper's spectral example.
"""
from __future__ import annotations

import numpy as np


def uniform_points(n: int, seed: int, dim: int = 2) -> np.ndarray:
    """n x dim points uniform on the unit square/cube, row-major float64."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, dim)), dtype=np.float64)


def mixture_points(n: int, seed: int, n_comp: int = 50, sd: float = 0.02) -> np.ndarray:
    """n x 2 points from an equal-weight Gaussian mixture on [0, 1]^2."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_comp, 2))
    out = np.empty((n, 2))
    filled = 0
    while filled < n:
        k = n - filled
        comp = rng.integers(0, n_comp, size=k)
        pts = centres[comp] + sd * rng.standard_normal((k, 2))
        ok = np.all((pts >= 0.0) & (pts <= 1.0), axis=1)
        good = pts[ok]
        out[filled:filled + good.shape[0]] = good
        filled += good.shape[0]
    return np.ascontiguousarray(out)


def normals(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)


def smooth_field(X: np.ndarray, seed: int, s2: float = 1.0, ell: float = 0.05,
                 t2: float = 0.01, n_waves: int = 256) -> np.ndarray:
    """Smooth random response at the rows of X (see module docstring)."""
    rng = np.random.default_rng(seed)
    d = X.shape[1]
    w = rng.standard_normal((n_waves, d)) / ell
    b = rng.uniform(0.0, 2.0 * np.pi, size=n_waves)
    f = np.sqrt(2.0 * s2 / n_waves) * np.cos(X @ w.T + b).sum(axis=1)
    return f + np.sqrt(t2) * rng.standard_normal(X.shape[0])


def spectral_points(n_phase: int, n_wave: int, seed: int, t_range=(-15.0, 24.0), lam_range=(5600.0, 6650.0),
                    noise_sd=(0.005, 0.02)) -> np.ndarray:
    """Rows (t, w, v) on a phase x log-wavelength grid, the layout of the
    paper's example data (25 phases x 2691 wavelengths = 67,275
    observations): n_phase phases uniform on t_range (sorted), n_wave
    log-wavelengths w = log(lambda) equally spaced over lam_range (Angstrom),
    and per-observation noise variances v = sd^2 with sd uniform on noise_sd.
    Phase-major order: all wavelengths of the first phase, then the next."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(t_range[0], t_range[1], size=n_phase))
    w = np.log(np.linspace(lam_range[0], lam_range[1], n_wave))
    sd = rng.uniform(noise_sd[0], noise_sd[1], size=n_phase * n_wave)
    out = np.empty((n_phase * n_wave, 3))
    out[:, 0] = np.repeat(t, n_wave)
    out[:, 1] = np.tile(w, n_phase)
    out[:, 2] = sd * sd
    return out


def batch_sizes(nb: int, seed: int, lo: int = 256, hi: int = 4096) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=nb).astype(np.int64)


# Workload definitions: sizes, covariance family and parameters of the five
# synthetic workloads (kernel codes: 0 exponential, 1 Matern-3/2, 2 Matern-5/2).
WORKLOADS = {
    "exp_n1024": dict(n=1024, kernel=0, sigma2=1.0, rho=0.1, tau2=0.1, seed=1, points="uniform"),
    "matern32_n16384": dict(n=16384, m=4096, kernel=1, sigma2=1.0, rho=0.05, tau2=0.01, seed=2,
                            points="uniform"),
    "exp_n32768": dict(n=32768, kernel=0, sigma2=1.0, rho=0.1, tau2=0.1, seed=4, points="uniform"),
    "matern32_mix_n67275": dict(n=67275, kernel=1, sigma2=1.0, rho=0.05, tau2=0.01, seed=5,
                                points="mixture"),
}


def points_for(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w["points"] == "mixture":
        return mixture_points(w["n"], w["seed"])
    return uniform_points(w["n"], w["seed"])
