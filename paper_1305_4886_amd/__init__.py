"""MI355X (gfx950) Gaussian-process likelihood library -- Python binding.

Thin ctypes layer over ``libgpmi.so`` (C ABI in ``include/gpmi.h``): argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; PyTorch provides device memory and the stream.  There is no CPU
fallback: if the library is not built or no GPU is present, calls raise.

Matrices are column-major.  A matrix with n rows and leading dimension ld is
held in a torch tensor ``S`` of shape ``(ncols, ld)`` whose row j is column j
(``colmajor(S, n)`` returns the (n x ncols) matrix view).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpmi.so")
TUNING_TABLE = os.path.join(_HERE, "tuning.txt")  # written by paper_1305_4886_amd/tune.py

GP_EXP, GP_MATERN32, GP_MATERN52, GP_SEP_MATERN2 = 0, 1, 2, 3
GP_FP64, GP_FP32_TRAIL, GP_BF16_TRAIL = 0, 1, 2
GP_NOTRANS, GP_TRANS = 0, 1
(GP_OP_POTRF, GP_OP_TRSV, GP_OP_TRSM, GP_OP_LOGLIK, GP_OP_LOGLIK_GRAD, GP_OP_KRIGE,
 GP_OP_BATCHED, GP_OP_MORTON, GP_OP_KRIGE_COV, GP_OP_TRMM, GP_OP_SIMULATE) = range(11)

KERNELS = {"exp": GP_EXP, "exponential": GP_EXP, "matern32": GP_MATERN32, "matern52": GP_MATERN52,
           "sep_matern2": GP_SEP_MATERN2}
PRECS = {"fp64": GP_FP64, "fp32": GP_FP32_TRAIL, "bf16": GP_BF16_TRAIL}

EXPORTED = ["gp_create", "gp_destroy", "gp_set_stream", "gp_set_options", "gp_get_options",
            "gp_strerror", "gp_profile", "gp_profile_read", "gp_workspace_size", "gp_cov_build", "gp_cross_cov_build", "gp_potrf",
            "gp_trsv", "gp_trsm", "gp_loglik", "gp_loglik_grad", "gp_krige", "gp_loglik_batched",
            "gp_morton_order", "gp_tune_potrf", "gp_tune_batched", "gp_loglik_noalloc", "gp_krige_cov",
            "gp_trmm", "gp_simulate", "gp_tune_save", "gp_tune_load", "gp_tune_clear", "gp_potrf_plan"]


class Theta(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("log_sigma2", ctypes.c_double),
                ("log_rho", ctypes.c_double), ("log_tau2", ctypes.c_double),
                ("log_rho2", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int32), ("lookahead", ctypes.c_int32), ("band", ctypes.c_int32),
                ("ir_max_iter", ctypes.c_int32), ("ir_tol", ctypes.c_double),
                ("reorder", ctypes.c_int32), ("panel_cus", ctypes.c_int32),
                ("fused_panel", ctypes.c_int32), ("batch_grid", ctypes.c_int32),
                ("fail_inject", ctypes.c_int32), ("bf16_split", ctypes.c_int32),
                ("syrk_slab", ctypes.c_int32), ("batch_tile", ctypes.c_int32), ("tail_nb", ctypes.c_int32)]


class GPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gpmi error %d: %s" % (code, msg))
        self.code = code


class NotPositiveDefinite(RuntimeError):
    def __init__(self, info):
        super().__init__("covariance not positive definite at column %d" % info)
        self.info = int(info)


_lib = None
_lock = threading.Lock()


def lib():
    """Load libgpmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgpmi.so is not built; run `python -m paper_1305_4886_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        L.gp_create.argtypes = [ctypes.POINTER(vp), vp]
        L.gp_destroy.argtypes = [vp]
        L.gp_set_stream.argtypes = [vp, vp]
        L.gp_set_options.argtypes = [vp, ctypes.POINTER(Options)]
        L.gp_get_options.argtypes = [vp, ctypes.POINTER(Options)]
        L.gp_profile.argtypes = [vp, ctypes.c_int]
        L.gp_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.gp_strerror.argtypes = [ctypes.c_int]
        L.gp_strerror.restype = ctypes.c_char_p
        L.gp_workspace_size.argtypes = [vp, ctypes.c_int, i64, i64, ctypes.c_int, ctypes.POINTER(sz)]
        L.gp_cov_build.argtypes = [vp, Theta, i64, i32, vp, vp, i64]
        L.gp_cross_cov_build.argtypes = [vp, Theta, i64, i64, i32, vp, vp, vp, i64]
        L.gp_potrf.argtypes = [vp, ctypes.c_int, i64, vp, i64, vp, vp, sz]
        L.gp_tune_potrf.argtypes = [vp, ctypes.c_int, i64, vp, i64, ctypes.POINTER(i32), i32, ctypes.POINTER(i32),
                                    i32, vp, ctypes.POINTER(dbl), vp, sz]
        L.gp_trsv.argtypes = [vp, ctypes.c_int, i64, vp, i64, vp, vp, sz]
        L.gp_trsm.argtypes = [vp, ctypes.c_int, i64, i64, vp, i64, vp, i64, vp, sz]
        L.gp_loglik.argtypes = [vp, Theta, ctypes.c_int, i64, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, sz]
        L.gp_loglik_noalloc.argtypes = [vp, Theta, ctypes.c_int, i64, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp]
        L.gp_loglik_grad.argtypes = [vp, Theta, ctypes.c_int, i64, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp,
                                     vp, vp, sz]
        L.gp_krige.argtypes = [vp, Theta, i64, i64, i32, vp, vp, vp, i64, vp, dbl, vp, vp, i32, vp, sz]
        L.gp_tune_save.argtypes = [vp, ctypes.c_char_p]
        L.gp_tune_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i32)]
        L.gp_tune_clear.argtypes = [vp]
        L.gp_potrf_plan.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        L.gp_krige_cov.argtypes = [vp, Theta, i64, i64, i32, vp, vp, vp, i64, i32, vp, i64, vp, sz]
        L.gp_trmm.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz]
        L.gp_simulate.argtypes = [vp, Theta, i64, i64, i32, vp, vp, vp, i64, vp, dbl, i32, i64, vp, i64, vp, i64,
                                  vp, i64, vp, vp, sz]
        L.gp_loglik_batched.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, sz]
        L.gp_morton_order.argtypes = [vp, i64, i32, vp, vp, vp, sz]
        L.gp_tune_batched.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32), i32, ctypes.POINTER(dbl), vp, sz]
        _lib = L
    return _lib


def check(rc):
    if rc != 0:
        raise GPError(rc, lib().gp_strerror(rc).decode())


def theta(kernel, sigma2=None, rho=None, tau2=None, log=None, rho2=None):
    """Theta from natural parameters or from log = (log s2, log rho, log t2
    [, log rho_w]); rho2 / the fourth log entry is the log-wavelength range of
    the separable family (GP_SEP_MATERN2)."""
    k = KERNELS.get(kernel, kernel) if isinstance(kernel, str) else int(kernel)
    lr2 = 0.0
    if log is not None:
        vals = [float(v) for v in log]
        ls, lr, lt = vals[:3]
        if len(vals) > 3:
            lr2 = vals[3]
    else:
        ls = math.log(sigma2) if sigma2 > 0 else -math.inf
        lr = math.log(rho)
        lt = math.log(tau2) if tau2 > 0 else -math.inf
        if rho2 is not None:
            lr2 = math.log(rho2)
    return Theta(k, ls, lr, lt, lr2)


def _torch():
    import torch
    return torch


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """A library handle bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        torch = _torch()
        self._h = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib().gp_create(ctypes.byref(self._h), ctypes.c_void_p(s.cuda_stream)))
        self.stream = s
        # the tuned choices measured on this architecture and shipped with the
        # package (entries of other architectures are skipped by the library)
        if os.path.exists(TUNING_TABLE):
            self.tune_load(TUNING_TABLE)

    def __del__(self):
        try:
            if self._h:
                lib().gp_destroy(self._h)
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def set_stream(self, s):
        check(lib().gp_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))
        self.stream = s

    def options(self):
        o = Options()
        check(lib().gp_get_options(self._h, ctypes.byref(o)))
        return o

    def set_options(self, **kw):
        o = self.options()
        for k, v in kw.items():
            setattr(o, k, v)
        check(lib().gp_set_options(self._h, ctypes.byref(o)))

    def tune_save(self, path):
        check(lib().gp_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path):
        n = ctypes.c_int32(0)
        check(lib().gp_tune_load(self._h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def tune_clear(self):
        check(lib().gp_tune_clear(self._h))

    def potrf_plan(self, n, prec=GP_FP64):
        """(panel width, reserved CUs, K-slab, tail panel width) the factorisation of an
        n x n matrix would use."""
        v = [ctypes.c_int32(0) for _ in range(4)]
        check(lib().gp_potrf_plan(self._h, int(prec), int(n), *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def tune_reset(self):
        """Back to the shipped table (or an empty one)."""
        self.tune_clear()
        if os.path.exists(TUNING_TABLE):
            self.tune_load(TUNING_TABLE)

    def profile(self, enable=True):
        check(lib().gp_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(launches, milliseconds, algorithmic flops, algorithmic bytes) of trailing updates
        since the last read."""
        out = (ctypes.c_double * 4)()
        check(lib().gp_profile_read(self._h, out))
        return int(out[0]), float(out[1]), float(out[2]), float(out[3])

    def tune_potrf(self, n, prec=GP_FP64, nb=(256, 384, 512, 768, 1024), panel_cus=(0, 8, 16)):
        """Time gp_potrf over (nb, panel_cus) -- and, in FP64, both trailing-update tile shapes --
        on a synthetic matrix of order n; keep the fastest in this handle's options and in its
        tuning table for n's size bucket.  Returns {(nb, panel_cus): ms} (-1: did not fit)."""
        torch = _torch()
        nb = [int(v) for v in nb]
        cus = [int(v) for v in panel_cus]
        saved = self.options()
        need = 0
        for v in nb:
            self.set_options(nb=v)
            b = ctypes.c_size_t()
            check(lib().gp_workspace_size(self._h, GP_OP_POTRF, n, 0, prec, ctypes.byref(b)))
            need = max(need, b.value)
        self.set_options(nb=saved.nb)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        A = colmajor_storage(n)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        nb_a = (ctypes.c_int32 * len(nb))(*nb)
        cu_a = (ctypes.c_int32 * len(cus))(*cus)
        ms = (ctypes.c_double * (len(nb) * len(cus)))()
        check(lib().gp_tune_potrf(self._h, prec, n, _ptr(A), A.shape[1], nb_a, len(nb), cu_a, len(cus),
                                  _ptr(info), ms, _ptr(ws), ws.numel()))
        return {(nb[a], cus[b]): ms[a * len(cus) + b] for a in range(len(nb)) for b in range(len(cus))}

    def tune_batched(self, X, y, thetas, sizes, grids=None, tiles=None):
        """Time gp_loglik_batched over candidate schedules and keep the fastest in this
        handle's options and tuning table.  Candidates are (batch_grid, batch_tile) pairs:
        `grids` (-1 level-synchronous, 0 one persistent workgroup per compute unit, > 0 that
        many) with `tiles` (64 / 128 / 0 automatic, one per grid; None: every grid keeps the
        options' tile).  Default: the level-synchronous launches, and one workgroup per
        compute unit and twice that with each tile edge.  Returns {(grid, tile): ms}
        (-1: did not fit)."""
        torch = _torch()
        import numpy as np
        X, y = _f64(X), _f64(y)
        nb = len(sizes)
        sizes = np.asarray(sizes, dtype=np.int64)
        if grids is None:
            ncu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
            grids = (-1, 0, 0, 2 * ncu, 2 * ncu)
            tiles = (0, 64, 128, 64, 128)
        grids = [int(g) for g in grids]
        tiles = [self.options().batch_tile] * len(grids) if tiles is None else [int(v) for v in tiles]
        if len(tiles) != len(grids):
            raise ValueError("one tile per grid candidate")
        x_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        c_off = np.concatenate([[0], np.cumsum(sizes * sizes)[:-1]]).astype(np.int64)
        th_arr = (Theta * nb)(*thetas)
        saved = self.options()
        self.set_options(batch_grid=1)  # persistent: the workspace query then covers every schedule and tile
        ws = self.workspace(GP_OP_BATCHED, int(sizes.max()), nb)
        self.set_options(batch_grid=saved.batch_grid)
        C_pool = torch.empty(max(int((sizes * sizes).sum()), 1), dtype=torch.float64, device="cuda")
        out3 = torch.empty(3 * nb, dtype=torch.float64, device="cuda")
        info = torch.zeros(nb, dtype=torch.int32, device="cuda")
        cand = (ctypes.c_int32 * len(grids))(*grids)
        tcand = (ctypes.c_int32 * len(grids))(*tiles)
        ms = (ctypes.c_double * len(grids))()
        check(lib().gp_tune_batched(self._h, nb, ctypes.cast(th_arr, ctypes.c_void_p),
                                    sizes.ctypes.data_as(ctypes.c_void_p), x_off.ctypes.data_as(ctypes.c_void_p),
                                    c_off.ctypes.data_as(ctypes.c_void_p), X.shape[1], _ptr(X), _ptr(y),
                                    _ptr(C_pool), _ptr(out3), _ptr(info), cand, tcand, len(grids), ms, _ptr(ws),
                                    ws.numel()))
        return {(grids[c], tiles[c]): ms[c] for c in range(len(grids))}

    def workspace(self, op, n, m=0, prec=GP_FP64):
        torch = _torch()
        b = ctypes.c_size_t()
        check(lib().gp_workspace_size(self._h, op, n, m, prec, ctypes.byref(b)))
        return torch.empty(max(b.value, 256), dtype=torch.uint8, device="cuda")


_handles = {}


def handle():
    """Per-(device, stream) cached handle on torch's current stream."""
    torch = _torch()
    s = torch.cuda.current_stream()
    key = (torch.cuda.current_device(), s.cuda_stream)
    h = _handles.get(key)
    if h is None:
        h = Handle(s)
        _handles[key] = h
    return h


def colmajor_storage(n, ncols=None, ld=None, dtype=None):
    """Device storage for an n x ncols column-major matrix with leading dim ld
    (default: n rounded up to even, so that every column starts on a 16-byte
    boundary and the factorisation's products take their 16-byte copies)."""
    torch = _torch()
    ncols = n if ncols is None else ncols
    ld = max(n + (n & 1), 1) if ld is None else ld
    return torch.zeros((max(ncols, 1), ld), dtype=dtype or torch.float64, device="cuda")


def colmajor(S, n):
    """(n x ncols) matrix view of column-major storage S (shape (ncols, ld))."""
    return S[:, :n].T


def _f64(t):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_contiguous():
        t = t.to(dtype=torch.float64).contiguous()
    return t


# ----------------------------------------------------------------------------
# Entry points (same names as the C ABI, without the gp_ prefix)
# ----------------------------------------------------------------------------
def cov_build(X, th, S=None):
    X = _f64(X)
    n, d = X.shape
    if S is None:
        S = colmajor_storage(n)
    check(lib().gp_cov_build(handle().ptr, th, n, d, _ptr(X), _ptr(S), S.shape[1]))
    return S


def cross_cov_build(X, Xs, th, S=None):
    X, Xs = _f64(X), _f64(Xs)
    n, d = X.shape
    m = Xs.shape[0]
    if S is None:
        S = colmajor_storage(n, m)
    check(lib().gp_cross_cov_build(handle().ptr, th, n, m, d, _ptr(X), _ptr(Xs), _ptr(S), S.shape[1]))
    return S


def potrf(S, n, prec=GP_FP64, ws=None):
    """In-place lower Cholesky of the column-major matrix in S; returns device info."""
    torch = _torch()
    h = handle()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_POTRF, n, 0, prec)
    check(lib().gp_potrf(h.ptr, prec, n, _ptr(S), S.shape[1], _ptr(info), _ptr(ws), ws.numel()))
    return info


def trsv(S, n, x, trans=False, ws=None):
    h = handle()
    ws = ws if ws is not None else h.workspace(GP_OP_TRSV, n)
    check(lib().gp_trsv(h.ptr, GP_TRANS if trans else GP_NOTRANS, n, _ptr(S), S.shape[1], _ptr(x),
                        _ptr(ws), ws.numel()))
    return x


def trsm(S, n, B, trans=False, ws=None):
    """B: column-major storage (nrhs, ldb) of an n x nrhs matrix, solved in place."""
    h = handle()
    nrhs = B.shape[0]
    ws = ws if ws is not None else h.workspace(GP_OP_TRSM, n, nrhs)
    check(lib().gp_trsm(h.ptr, GP_TRANS if trans else GP_NOTRANS, n, nrhs, _ptr(S), S.shape[1], _ptr(B),
                        B.shape[1], _ptr(ws), ws.numel()))
    return B


def loglik(X, y, th, prec=GP_FP64, mu=None, S=None, want_alpha=False, ws=None):
    """Returns dict with device tensors out3 = [loglik, logdet, q], info, S (factor), alpha, ir."""
    torch = _torch()
    X, y = _f64(X), _f64(y)
    n, d = X.shape
    h = handle()
    S = S if S is not None else colmajor_storage(n)
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ir = torch.zeros(3, dtype=torch.float64, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda") if want_alpha else None
    mu_t = None if mu is None else _f64(torch.as_tensor(mu, dtype=torch.float64, device="cuda").expand(n).contiguous())
    ws = ws if ws is not None else h.workspace(GP_OP_LOGLIK, n, 0, prec)
    check(lib().gp_loglik(h.ptr, th, prec, n, d, _ptr(X), _ptr(y), _ptr(mu_t), _ptr(S), S.shape[1],
                          _ptr(out3), _ptr(alpha), _ptr(info), _ptr(ir), _ptr(ws), ws.numel()))
    return dict(out3=out3, info=info, S=S, alpha=alpha, ir=ir)


def loglik_noalloc(X, y, th, prec=GP_FP64, mu=None, S=None, want_alpha=False):
    """gp_loglik_noalloc: as loglik(), with the library's static workspace
    instead of a caller-allocated one (the outputs are still allocated here
    unless S is given)."""
    torch = _torch()
    X, y = _f64(X), _f64(y)
    n, d = X.shape
    h = handle()
    S = S if S is not None else colmajor_storage(n)
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ir = torch.zeros(3, dtype=torch.float64, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda") if want_alpha else None
    mu_t = None if mu is None else _f64(torch.as_tensor(mu, dtype=torch.float64, device="cuda").expand(n).contiguous())
    check(lib().gp_loglik_noalloc(h.ptr, th, prec, n, d, _ptr(X), _ptr(y), _ptr(mu_t), _ptr(S), S.shape[1],
                                  _ptr(out3), _ptr(alpha), _ptr(info), _ptr(ir)))
    return dict(out3=out3, info=info, S=S, alpha=alpha, ir=ir)


def loglik_grad(X, y, th, prec=GP_FP64, mu=None, S=None, want_alpha=False, ws=None):
    torch = _torch()
    X, y = _f64(X), _f64(y)
    n, d = X.shape
    h = handle()
    S = S if S is not None else colmajor_storage(n)
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    grad3 = torch.empty(4 if th.kind == GP_SEP_MATERN2 else 3, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ir = torch.zeros(3, dtype=torch.float64, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda") if want_alpha else None
    mu_t = None if mu is None else _f64(torch.as_tensor(mu, dtype=torch.float64, device="cuda").expand(n).contiguous())
    ws = ws if ws is not None else h.workspace(GP_OP_LOGLIK_GRAD, n, 0, prec)
    check(lib().gp_loglik_grad(h.ptr, th, prec, n, d, _ptr(X), _ptr(y), _ptr(mu_t), _ptr(S), S.shape[1],
                               _ptr(out3), _ptr(grad3), _ptr(alpha), _ptr(info), _ptr(ir), _ptr(ws),
                               ws.numel()))
    return dict(out3=out3, grad=grad3, info=info, S=S, alpha=alpha, ir=ir)


def krige(X, Xs, S, alpha, th, mu=0.0, include_nugget=False, ws=None):
    torch = _torch()
    X, Xs = _f64(X), _f64(Xs)
    n, d = X.shape
    m = Xs.shape[0]
    h = handle()
    mean = torch.empty(m, dtype=torch.float64, device="cuda")
    var = torch.empty(m, dtype=torch.float64, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_KRIGE, n, m)
    check(lib().gp_krige(h.ptr, th, n, m, d, _ptr(X), _ptr(Xs), _ptr(S), S.shape[1], _ptr(alpha),
                         float(mu), _ptr(mean), _ptr(var), 1 if include_nugget else 0, _ptr(ws), ws.numel()))
    return mean, var


def krige_cov(X, Xs, S_data, th, include_nugget=False, out=None, ws=None):
    """gp_krige_cov: the m x m prediction covariance of the new points Xs given
    the data X with factor storage S_data (X = None: the prior covariance).
    Returns column-major storage P (shape (m, m), element (i, j) at P[j, i]),
    lower triangle filled."""
    torch = _torch()
    Xs = _f64(Xs)
    m, d = Xs.shape
    n = 0 if X is None else X.shape[0]
    X = None if X is None else _f64(X)
    h = handle()
    P = out if out is not None else colmajor_storage(m)
    ws = ws if ws is not None else h.workspace(GP_OP_KRIGE_COV, n, m)
    ldl = S_data.shape[1] if S_data is not None else 1
    check(lib().gp_krige_cov(h.ptr, th, n, m, d, _ptr(X), _ptr(Xs), _ptr(S_data), ldl,
                             1 if include_nugget else 0, _ptr(P), P.shape[1], _ptr(ws), ws.numel()))
    return P


def trmm(S, E, ws=None):
    """gp_trmm: L E for the lower factor in storage S (shape (n, ld)) and E in
    column-major storage of shape (nrhs, n); returns storage of shape (nrhs, n)."""
    torch = _torch()
    E = _f64(E)
    nrhs, n = E.shape
    h = handle()
    out = torch.empty((nrhs, n), dtype=torch.float64, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_TRMM, n, nrhs)
    check(lib().gp_trmm(h.ptr, n, nrhs, _ptr(S), S.shape[1], _ptr(E), max(n, 1), _ptr(out), max(n, 1),
                        _ptr(ws), ws.numel()))
    return out


def simulate(Xs, th, eps, X=None, S_data=None, alpha=None, mu=0.0, include_nugget=False, S=None, ws=None):
    """gp_simulate: realizations mean + L_S eps at the new points Xs,
    unconditional (X None) or conditional on the data (X, its factor storage
    S_data and alpha from loglik).  eps: column-major storage of shape
    (nreal, m) (realization r is eps[r]).  Returns dict(out (nreal, m), info,
    S (the factor L_S, storage (m, m)))."""
    torch = _torch()
    Xs = _f64(Xs)
    eps = _f64(eps)
    m, d = Xs.shape
    nreal = eps.shape[0]
    assert eps.shape[1] == m
    n = 0 if X is None else X.shape[0]
    X = None if X is None else _f64(X)
    h = handle()
    S = S if S is not None else colmajor_storage(m)
    out = torch.empty((nreal, m), dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_SIMULATE, n, m)
    ldl = S_data.shape[1] if S_data is not None else 1
    check(lib().gp_simulate(h.ptr, th, n, m, d, _ptr(X), _ptr(Xs), _ptr(S_data), ldl, _ptr(alpha), float(mu),
                            1 if include_nugget else 0, nreal, _ptr(eps), max(m, 1), _ptr(out), max(m, 1),
                            _ptr(S), S.shape[1], _ptr(info), _ptr(ws), ws.numel()))
    return dict(out=out, info=info, S=S)


def loglik_batched(X, y, thetas, sizes, x_off=None, C_pool=None, ws=None):
    """Independent problems b: points X[x_off[b] : x_off[b] + sizes[b]]."""
    torch = _torch()
    import numpy as np
    X, y = _f64(X), _f64(y)
    nb = len(sizes)
    sizes = np.asarray(sizes, dtype=np.int64)
    x_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if x_off is None else \
        np.asarray(x_off, dtype=np.int64)
    c_off = np.concatenate([[0], np.cumsum(sizes * sizes)[:-1]]).astype(np.int64)
    th_arr = (Theta * nb)(*thetas)
    h = handle()
    if C_pool is None:
        C_pool = torch.empty(int((sizes * sizes).sum()), dtype=torch.float64, device="cuda")
    out3 = torch.empty(3 * nb, dtype=torch.float64, device="cuda")
    info = torch.zeros(nb, dtype=torch.int32, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_BATCHED, int(sizes.max()), nb)
    check(lib().gp_loglik_batched(h.ptr, nb, ctypes.cast(th_arr, ctypes.c_void_p),
                                  sizes.ctypes.data_as(ctypes.c_void_p), x_off.ctypes.data_as(ctypes.c_void_p),
                                  c_off.ctypes.data_as(ctypes.c_void_p), X.shape[1], _ptr(X), _ptr(y),
                                  _ptr(C_pool), _ptr(out3), _ptr(info), _ptr(ws), ws.numel()))
    return dict(out3=out3.view(nb, 3), info=info, C_pool=C_pool)


def morton_order(X, ws=None):
    torch = _torch()
    X = _f64(X)
    n, d = X.shape
    h = handle()
    perm = torch.empty(n, dtype=torch.int64, device="cuda")
    ws = ws if ws is not None else h.workspace(GP_OP_MORTON, n)
    check(lib().gp_morton_order(h.ptr, n, d, _ptr(X), _ptr(perm), _ptr(ws), ws.numel()))
    return perm


def _loglik_function():
    torch = _torch()

    class LogLik(torch.autograd.Function):
        """Marginal log-likelihood as a differentiable function of
        log_theta = (log sigma^2, log rho, log tau^2).  The forward pass runs
        gp_loglik, or gp_loglik_grad when log_theta needs a gradient (the
        adjoint is formed in the same pass); backward scales that gradient."""

        @staticmethod
        def forward(ctx, log_theta, X, y, kind, prec, mu):
            th = theta(kind, log=[float(v) for v in log_theta.detach().cpu()])
            if ctx.needs_input_grad[0]:
                r = loglik_grad(X, y, th, prec, mu)
                g = r["grad"]
            else:
                r = loglik(X, y, th, prec, mu)
                g = None
            info = int(r["info"].item())
            if info > 0:
                raise NotPositiveDefinite(info)
            ctx.save_for_backward(g if g is not None else torch.zeros(3, dtype=torch.float64, device="cuda"))
            return r["out3"][0].clone().to(log_theta.device)

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return (gout * g).to(gout.device), None, None, None, None, None

    return LogLik


_LogLik = None


def log_likelihood(X, y, log_theta, kernel=GP_EXP, prec=GP_FP64, mu=None):
    """Differentiable loglik: a 0-d tensor whose backward gives d loglik / d log_theta."""
    global _LogLik
    if _LogLik is None:
        _LogLik = _loglik_function()
    k = KERNELS.get(kernel, kernel) if isinstance(kernel, str) else int(kernel)
    return _LogLik.apply(log_theta, X, y, k, prec, mu)
