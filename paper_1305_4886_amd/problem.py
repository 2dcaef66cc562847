"""Maximum-likelihood fitting and the analysis steps that follow it.

``KrigeProblem`` is this library's form of the problem object the paper's
package builds its standard analyses on (Section 2.3.3): it holds the data
and the covariance family, the current parameter vector, and flags saying
which derived objects (the Cholesky factor L, alpha = C^{-1}(y - mu), the
last log-likelihood and gradient) are up to date for it, so that nothing is
recomputed while the parameters are unchanged.  On top of the GPU calls it
runs the optimisation of the log-likelihood (Section 1: maximised over theta
to find the MLE; the paper's example uses L-BFGS-B, Section 4.3), prediction
with standard errors, the full prediction covariance and simulation of
realizations conditional on the data at the estimate.

Parameters are log_theta = (log sigma^2, log rho, log tau^2), with a fourth
entry log rho_w for the separable spectral family (kernel 3).  Every
numerical step runs in the GPU library; this module only keeps state and
drives scipy's optimiser over the values and gradients the library returns.
"""
from __future__ import annotations

import math

import numpy as np

from . import (GP_FP64, GP_OP_LOGLIK, GP_OP_LOGLIK_GRAD, KERNELS, NotPositiveDefinite, colmajor_storage,
               handle, theta)
from . import krige as _krige
from . import krige_cov as _krige_cov
from . import loglik as _loglik
from . import loglik_grad as _loglik_grad
from . import simulate as _simulate


class KrigeProblem:
    """Data X (n x dim) and y (n) on the GPU, covariance family `kernel`,
    constant mean mu, trailing-update precision `prec` for the likelihood
    evaluations of the optimiser (the factor used for prediction is always
    the FP64 one)."""

    def __init__(self, X, y, kernel, log_theta=None, mu=0.0, prec=GP_FP64):
        import torch

        self.torch = torch
        self.X = torch.as_tensor(X, dtype=torch.float64, device="cuda").contiguous()
        self.y = torch.as_tensor(y, dtype=torch.float64, device="cuda").contiguous()
        self.n, self.dim = self.X.shape
        self.kind = KERNELS.get(kernel, kernel) if isinstance(kernel, str) else int(kernel)
        self.mu = float(mu)
        self.prec = prec
        self.S = colmajor_storage(self.n)  # L (or C^{-1} after a gradient evaluation)
        h = handle()
        self._ws_l = {}
        self._ws_g = {}
        self._h = h
        self.theta = None if log_theta is None else np.asarray(log_theta, dtype=np.float64).copy()
        # up-to-date flags: what S and the cached values belong to
        self._S_holds = None      # ("factor", key) | ("inverse", key) | None
        self._alpha = None        # alpha for the factor in S
        self._ll = {}             # key -> (loglik, logdet, q)
        self._grad = {}           # key -> gradient
        self.evaluations = {"loglik": 0, "loglik_grad": 0}

    # ---- bookkeeping ------------------------------------------------------
    @staticmethod
    def _key(log_theta, prec):
        return (tuple(float(v) for v in np.asarray(log_theta, dtype=np.float64).reshape(-1)), int(prec))

    def _ws(self, grad, prec):
        cache = self._ws_g if grad else self._ws_l
        if prec not in cache:
            cache[prec] = self._h.workspace(GP_OP_LOGLIK_GRAD if grad else GP_OP_LOGLIK, self.n, 0, prec)
        return cache[prec]

    def _th(self, log_theta):
        return theta(self.kind, log=[float(v) for v in np.asarray(log_theta).reshape(-1)])

    @staticmethod
    def _check(r):
        info = int(r["info"].item())
        if info != 0:
            raise NotPositiveDefinite(info)

    # ---- the likelihood ---------------------------------------------------
    def log_density(self, log_theta=None, prec=None):
        """Marginal log-likelihood (Section 1) at log_theta (default: the
        current parameters); evaluated only if not already known there."""
        lt = self.theta if log_theta is None else log_theta
        prec = self.prec if prec is None else prec
        key = self._key(lt, prec)
        if key in self._ll:
            return self._ll[key][0]
        want_alpha = prec == GP_FP64
        r = _loglik(self.X, self.y, self._th(lt), prec=prec, mu=self.mu, S=self.S, ws=self._ws(False, prec),
                    want_alpha=want_alpha)
        self.evaluations["loglik"] += 1
        self._check(r)
        self._ll[key] = tuple(float(v) for v in r["out3"].cpu().numpy())
        # a mixed-precision factor belongs to the reordered points: not reusable for prediction
        self._S_holds = ("factor", key) if want_alpha else None
        self._alpha = r["alpha"] if want_alpha else None
        return self._ll[key][0]

    def log_density_grad(self, log_theta=None, prec=None):
        """(loglik, gradient with respect to log_theta), evaluated once per
        parameter vector by the adjoint (gp_loglik_grad).  S then holds C^{-1}
        and the factor must be rebuilt before prediction."""
        lt = self.theta if log_theta is None else log_theta
        prec = self.prec if prec is None else prec
        key = self._key(lt, prec)
        if key in self._grad:
            return self._ll[key][0], self._grad[key].copy()
        r = _loglik_grad(self.X, self.y, self._th(lt), prec=prec, mu=self.mu, S=self.S, ws=self._ws(True, prec))
        self.evaluations["loglik_grad"] += 1
        self._check(r)
        self._ll[key] = tuple(float(v) for v in r["out3"].cpu().numpy())
        self._grad[key] = r["grad"].cpu().numpy().copy()
        self._S_holds = ("inverse", key)
        self._alpha = None
        return self._ll[key][0], self._grad[key].copy()

    def optimize(self, log_theta0=None, bounds=None, method="L-BFGS-B", options=None):
        """Maximise the log-likelihood over log_theta with scipy's L-BFGS-B on
        the library's value and adjoint gradient.  bounds: (lo, hi) pairs in
        log coordinates (None entries unbounded).  Sets and returns the
        estimate; the scipy result is kept in self.opt_result."""
        from scipy.optimize import minimize

        x0 = np.asarray(self.theta if log_theta0 is None else log_theta0, dtype=np.float64).reshape(-1)

        def f(t):
            try:
                ll, g = self.log_density_grad(t)
            except NotPositiveDefinite:
                return math.inf, np.zeros(x0.size)
            return -ll, -g

        res = minimize(f, x0, jac=True, method=method, bounds=bounds,
                       options=dict({"maxiter": 200, "gtol": 1e-8, "ftol": 1e-14}, **(options or {})))
        self.opt_result = res
        self.theta = np.asarray(res.x, dtype=np.float64).copy()
        return self.theta

    # ---- analyses at the current parameters ------------------------------------
    def _ensure_factor(self):
        """S holds the FP64 factor of C(theta) and alpha is known."""
        key = self._key(self.theta, GP_FP64)
        if self._S_holds == ("factor", key) and self._alpha is not None:
            return
        self._ll.pop(key, None)
        self.log_density(self.theta, prec=GP_FP64)

    def predict(self, Xs, se=True, include_nugget=False):
        """Kriging mean (and standard errors) at the new points Xs."""
        self._ensure_factor()
        Xs = self.torch.as_tensor(Xs, dtype=self.torch.float64, device="cuda").contiguous()
        mean, var = _krige(self.X, Xs, self.S, self._alpha, self._th(self.theta), mu=self.mu,
                           include_nugget=include_nugget)
        return (mean, var.clamp_min(0.0).sqrt()) if se else mean

    def prediction_covariance(self, Xs, include_nugget=False):
        """The full m x m prediction covariance (column-major storage, lower)."""
        self._ensure_factor()
        Xs = self.torch.as_tensor(Xs, dtype=self.torch.float64, device="cuda").contiguous()
        return _krige_cov(self.X, Xs, self.S, self._th(self.theta), include_nugget=include_nugget)

    def simulate_realizations(self, Xs, r, post=True, include_nugget=False, seed=0):
        """r realizations of the latent process at Xs, conditional on the data
        (post=True) or from the prior; standard normals from a seeded torch
        generator.  Returns (out (r, m), info)."""
        torch = self.torch
        Xs = torch.as_tensor(Xs, dtype=torch.float64, device="cuda").contiguous()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        eps = torch.randn((r, Xs.shape[0]), dtype=torch.float64, device="cuda", generator=gen)
        if post:
            self._ensure_factor()
            res = _simulate(Xs, self._th(self.theta), eps, X=self.X, S_data=self.S, alpha=self._alpha, mu=self.mu,
                            include_nugget=include_nugget)
        else:
            res = _simulate(Xs, self._th(self.theta), eps, mu=self.mu, include_nugget=include_nugget)
        return res["out"], int(res["info"].item())
