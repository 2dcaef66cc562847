"""CPU FP64 oracle for the Gaussian-process likelihood path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never links, imports
or calls it, and it shares no code with the GPU library: the arithmetic lives
in ``gp_oracle.c`` (plain C, no BLAS), this file only marshals numpy arrays.

Parameters are ``theta = (log sigma^2, log rho, log tau^2)``; kernels are
0 = exponential, 1 = Matern-3/2, 2 = Matern-5/2 (Rasmussen-Williams scaling
sqrt(2 nu) d / rho), and 3 = the example's separable family (points
(t, w, v): product of Matern-2 correlations in t and w, random effect tau^2
shared by equal t, noise variance v on the diagonal; theta has a fourth
entry log rho_w and the gradient four components).  Matrices are numpy arrays in Fortran (column-major) order.

Parity unpinned: none -- every function here is pinned by ``tests/test_oracle_pins.py``
(closed forms, hand-derived factors, exact rational arithmetic, LAPACK, finite
differences and the sigma^2/tau^2 scale identity).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def build(force: bool = False) -> str:
    """Compile gp_oracle.c into liboracle.so (gcc, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_cov.argtypes = [ctypes.c_int, _dp, _i64, ctypes.c_int, _dp, _dp, _i64]
        L.orc_cross_cov.argtypes = [ctypes.c_int, _dp, _i64, _i64, ctypes.c_int, _dp, _dp, _dp, _i64]
        L.orc_potrf.argtypes = [_i64, _dp, _i64]
        L.orc_potrf.restype = _i64
        L.orc_trsv.argtypes = [ctypes.c_int, _i64, _dp, _i64, _dp]
        L.orc_logdet_q.argtypes = [_i64, _dp, _i64, _dp, _dp]
        L.orc_loglik.argtypes = [ctypes.c_int, _dp, _i64, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_loglik.restype = _i64
        L.orc_inv_lower.argtypes = [_i64, _dp, _i64, _dp, _i64]
        L.orc_loglik_grad.argtypes = [ctypes.c_int, _dp, _i64, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_loglik_grad.restype = _i64
        L.orc_krige.argtypes = [ctypes.c_int, _dp, _i64, _i64, ctypes.c_int, _dp, _dp, _dp, _i64,
                                _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.orc_krige_cov.argtypes = [ctypes.c_int, _dp, _i64, _i64, ctypes.c_int, _dp, _dp, _dp, _i64,
                                    ctypes.c_int, _dp, _i64]
        L.orc_trmm.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
        L.orc_simulate.argtypes = [ctypes.c_int, _dp, _i64, _i64, ctypes.c_int, _dp, _dp, _dp, _i64, _dp,
                                   ctypes.c_double, ctypes.c_int, _i64, _dp, _i64, _dp, _i64, _dp]
        L.orc_simulate.restype = _i64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _vec(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _th(theta):
    """(log sigma^2, log rho, log tau^2[, log rho_w]) -> 4 doubles (the fourth
    is read only by the separable family, kernel 3)."""
    t = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    if t.size not in (3, 4):
        raise ValueError("theta needs 3 (or 4 for kernel 3) values")
    return np.concatenate([t, np.zeros(4 - t.size)])


class NotPositiveDefinite(RuntimeError):
    def __init__(self, info):
        super().__init__("matrix not positive definite at column %d" % info)
        self.info = int(info)


def cov(kernel, theta, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    C = np.zeros((n, n), order="F")
    th = _th(theta)
    lib().orc_cov(kernel, _p(th), n, d, _p(X), _p(C), max(n, 1))
    return C


def cross_cov(kernel, theta, X, Xs):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    n, d = X.shape
    m = Xs.shape[0]
    Cs = np.zeros((n, m), order="F")
    th = _th(theta)
    lib().orc_cross_cov(kernel, _p(th), n, m, d, _p(X), _p(Xs), _p(Cs), max(n, 1))
    return Cs


def potrf(A):
    """Lower Cholesky factor of A (copy); returns (L, info). L is lower with zero upper."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    info = lib().orc_potrf(n, _p(A), max(n, 1))
    return np.tril(A), int(info)


def trsv(L, x, trans=False):
    L = np.asfortranarray(L, dtype=np.float64)
    x = np.array(x, dtype=np.float64, copy=True)
    n = L.shape[0]
    lib().orc_trsv(1 if trans else 0, n, _p(L), max(n, 1), _p(x))
    return x


def logdet_q(L, z):
    L = np.asfortranarray(L, dtype=np.float64)
    z = _vec(z)
    out = np.zeros(2)
    lib().orc_logdet_q(L.shape[0], _p(L), max(L.shape[0], 1), _p(z), _p(out))
    return float(out[0]), float(out[1])


def loglik(kernel, theta, X, y, mu=None, want=False):
    """Returns (loglik, logdet, q) or, with want=True, also (L, alpha)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    y = _vec(y)
    mu_a = None if mu is None else _vec(np.broadcast_to(mu, (n,)))
    L = np.zeros((n, n), order="F")
    out = np.zeros(3)
    alpha = np.zeros(n)
    th = _th(theta)
    info = lib().orc_loglik(kernel, _p(th), n, d, _p(X), _p(y), _p(mu_a), _p(L), _p(out), _p(alpha))
    if info:
        raise NotPositiveDefinite(info)
    res = (float(out[0]), float(out[1]), float(out[2]))
    if want:
        return res, np.tril(L), alpha
    return res


def loglik_grad(kernel, theta, X, y, mu=None):
    """Returns ((loglik, logdet, q), grad[3]) with grad w.r.t. log-parameters."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    y = _vec(y)
    mu_a = None if mu is None else _vec(np.broadcast_to(mu, (n,)))
    out = np.zeros(3)
    g = np.zeros(4)
    th = _th(theta)
    info = lib().orc_loglik_grad(kernel, _p(th), n, d, _p(X), _p(y), _p(mu_a), _p(out), _p(g))
    if info:
        raise NotPositiveDefinite(info)
    return (float(out[0]), float(out[1]), float(out[2])), (g if kernel == 3 else g[:3])


def inv_lower(L):
    L = np.asfortranarray(L, dtype=np.float64)
    n = L.shape[0]
    W = np.zeros((n, n), order="F")
    lib().orc_inv_lower(n, _p(L), max(n, 1), _p(W), max(n, 1))
    return W


def krige(kernel, theta, X, Xs, L, alpha, mu=0.0, include_nugget=False):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    L = np.asfortranarray(L, dtype=np.float64)
    n, d = X.shape
    m = Xs.shape[0]
    mean = np.zeros(m)
    var = np.zeros(m)
    th = _th(theta)
    lib().orc_krige(kernel, _p(th), n, m, d, _p(X), _p(Xs), _p(L), max(n, 1), _p(_vec(alpha)),
                    float(mu), 1 if include_nugget else 0, _p(mean), _p(var))
    return mean, var


def krige_cov(kernel, theta, X, Xs, L=None, include_nugget=False):
    """Full m x m prediction covariance (lower triangle filled, upper zero).
    X = None (or n = 0) gives the prior covariance of the new points."""
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    m, d = Xs.shape
    if X is None:
        X = np.zeros((0, d))
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    Lf = np.asfortranarray(L if L is not None else np.zeros((1, 1)), dtype=np.float64)
    S = np.zeros((m, m), order="F")
    th = _th(theta)
    lib().orc_krige_cov(kernel, _p(th), n, m, d, _p(X), _p(Xs), _p(Lf), max(n, 1),
                        1 if include_nugget else 0, _p(S), max(m, 1))
    return np.tril(S)


def trmm(L, B):
    """L B for lower-triangular L (only its lower triangle is read)."""
    L = np.asfortranarray(L, dtype=np.float64)
    B = np.array(B, dtype=np.float64, order="F", copy=True)
    if B.ndim == 1:
        B = B.reshape(-1, 1, order="F")
    n, r = B.shape
    lib().orc_trmm(n, r, _p(L), max(n, 1), _p(B), max(n, 1))
    return B


def simulate(kernel, theta, Xs, eps, X=None, L=None, alpha=None, mu=0.0, include_nugget=False,
             want_factor=False):
    """Realizations mean + L_S eps (m x nreal): unconditional when X is None,
    else conditional on the data whose factor L and alpha = C^{-1}(y - mu)
    are given.  Returns (out, info) or, with want_factor, (out, info, L_S)."""
    Xs = np.ascontiguousarray(Xs, dtype=np.float64)
    m, d = Xs.shape
    eps = np.asfortranarray(eps, dtype=np.float64)
    if eps.ndim == 1:
        eps = eps.reshape(-1, 1, order="F")
    r = eps.shape[1]
    if X is None:
        X = np.zeros((0, d))
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    Lf = np.asfortranarray(L if L is not None else np.zeros((1, 1)), dtype=np.float64)
    a = _vec(alpha) if alpha is not None else np.zeros(1)
    out = np.zeros((m, r), order="F")
    LS = np.zeros((m, m), order="F")
    th = _th(theta)
    info = lib().orc_simulate(kernel, _p(th), n, m, d, _p(X), _p(Xs), _p(Lf), max(n, 1), _p(a), float(mu),
                              1 if include_nugget else 0, r, _p(eps), max(m, 1), _p(out), max(m, 1), _p(LS))
    if want_factor:
        return out, int(info), LS
    return out, int(info)
