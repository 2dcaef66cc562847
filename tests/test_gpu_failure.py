"""Failure reporting and argument validation of the C ABI.

* Bounded waits that give up (the fused panel kernel's hand-over flags, the
  mailbox of the triangular solves) must surface as info = -1 with NaN
  outputs, never as a finite wrong result.  The condition is forced from the
  host (the fail_inject option raises the kernels' abort flags before they
  start), so every wait gives up at once and every kernel exits normally.
* A pivot failure (Section 5: no pivoting, a matrix that is not numerically
  positive definite fails) keeps its column in info even when other
  workgroups give up around it.
* The inverse-only mode of the panel kernel (kriging's band inverses) reads
  no flags, so stale flag words in a reused workspace cannot change kriging.
* Every entry point rejects bad arguments synchronously with the LAPACK-style
  code -k (k-th argument) or GP_ERR_NONFINITE / GP_ERR_WS_TOO_SMALL, and
  enqueues nothing.
"""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1305_4886_amd as gp  # noqa: E402
from paper_1305_4886_amd import synth  # noqa: E402

NONFINITE, WS_TOO_SMALL = -1001, -1002


def logth(s2, rho, t2):
    return np.array([math.log(s2), math.log(rho), math.log(t2)])


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


@pytest.fixture
def injected():
    h = gp.handle()
    saved = h.options()

    def set_(bits, **kw):
        h.set_options(fail_inject=bits, **kw)

    yield set_
    h.set_options(fail_inject=0, nb=saved.nb, lookahead=saved.lookahead, fused_panel=saved.fused_panel)


def problem(n, seed=3):
    X = synth.uniform_points(n, seed)
    y = synth.smooth_field(X, seed + 1, ell=0.1, t2=0.1)
    return X, y, gp.theta(0, log=logth(1.0, 0.1, 0.1))


@pytest.mark.parametrize("prec", [gp.GP_FP64, gp.GP_FP32_TRAIL])
def test_panel_giveup_reports_stall(injected, prec):
    n = 2048  # first panel: 768 (FP64) or 512 (FP32) columns, 8 or 12 concurrent workgroups
    X, y, th = problem(n)
    injected(1)
    r = gp.loglik(dev(X), dev(y), th, prec=prec, want_alpha=True)
    assert int(r["info"].item()) == -1
    assert np.all(np.isnan(r["out3"].cpu().numpy()))
    assert np.all(np.isnan(r["alpha"].cpu().numpy()))
    g = gp.loglik_grad(dev(X), dev(y), th, prec=prec)
    assert int(g["info"].item()) == -1
    assert np.all(np.isnan(g["grad"].cpu().numpy())) and np.all(np.isnan(g["out3"].cpu().numpy()))
    # the next call without the hook starts from fresh flags
    injected(0)
    r = gp.loglik(dev(X), dev(y), th, prec=prec)
    assert int(r["info"].item()) == 0 and np.all(np.isfinite(r["out3"].cpu().numpy()))


@pytest.mark.parametrize("n", [100, 4096])
def test_solve_giveup_reports_stall(injected, n):
    X, y, th = problem(n)
    injected(2)
    r = gp.loglik(dev(X), dev(y), th, want_alpha=True)
    assert int(r["info"].item()) == -1
    assert np.all(np.isnan(r["out3"].cpu().numpy()))
    assert np.all(np.isnan(r["alpha"].cpu().numpy()))
    m = gp.loglik(dev(X), dev(y), th, prec=gp.GP_FP32_TRAIL)
    assert int(m["info"].item()) == -1 and np.all(np.isnan(m["out3"].cpu().numpy()))
    injected(0)
    r = gp.loglik(dev(X), dev(y), th)
    assert int(r["info"].item()) == 0 and np.all(np.isfinite(r["out3"].cpu().numpy()))


@pytest.mark.parametrize("bad", [5, 300, 767, 1500])
def test_pivot_failure_keeps_its_column(orc, bad):
    """The failing workgroup records its column; the others give up around it."""
    n = 2048
    A = np.eye(n) * 2.0 + 0.01
    A[bad, bad] = -1.0
    S = gp.colmajor_storage(n)
    gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(A)))
    info = gp.potrf(S, n)
    _, info_o = orc.potrf(A)
    assert int(info.item()) == info_o == bad + 1


def test_krige_ignores_stale_panel_flags(orc):
    """Kriging on a reused workspace whose words look like raised abort flags
    and lowered hand-over flags (the layout of the panel kernel's flag area,
    which starts on a 256-byte boundary) must still match the oracle."""
    n, m = 1100, 300
    X = synth.uniform_points(n, 61)
    Xs = synth.uniform_points(m, 62)
    y = synth.smooth_field(X, 63, ell=0.1, t2=0.05)
    t = logth(1.0, 0.1, 0.05)
    th = gp.theta(1, log=t)
    r = gp.loglik(dev(X), dev(y), th, want_alpha=True)
    h = gp.handle()
    ws = h.workspace(gp.GP_OP_KRIGE, n, m)
    words = ws.view(torch.int32)
    g = torch.arange(words.numel(), device="cuda", dtype=torch.int64) % 64
    zero = torch.zeros_like(g, dtype=torch.bool)
    for k in range(1, 8):  # hand-over flag (k, k) of an 8-workgroup band: word 17 k
        zero |= g == (17 * k) % 64
    words.copy_(torch.where(zero, 0, 1).to(torch.int32))
    mean, var = gp.krige(dev(X), dev(Xs), r["S"], r["alpha"], th, ws=ws)
    (_, _, _), L, alpha = orc.loglik(1, t, X, y, want=True)
    mo, vo = orc.krige(1, t, X, Xs, L, alpha)
    mean, var = mean.cpu().numpy(), var.cpu().numpy()
    assert np.all(np.abs(mean - mo) <= 1e-10 * np.maximum(1.0, np.abs(mo)))
    assert np.all(np.abs(var - vo) <= 1e-10)


# ---------------------------------------------------------------------------
# argument validation (synchronous return codes, nothing enqueued)
# ---------------------------------------------------------------------------
def P(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.fixture
def ctx():
    n = 256
    X = dev(synth.uniform_points(n, 1))
    y = dev(synth.normals(n, 2))
    S = gp.colmajor_storage(n)
    out3 = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    grad = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    info = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    h = gp.handle()
    ws = h.workspace(gp.GP_OP_LOGLIK_GRAD, n)
    return dict(n=n, X=X, y=y, S=S, out3=out3, grad=grad, info=info, h=h, ws=ws)


def th_(kind=0, ls=0.0, lr=math.log(0.1), lt=math.log(0.1)):
    return gp.Theta(kind, ls, lr, lt)


def test_cov_build_arguments(ctx):
    L, c = gp.lib(), ctx
    h, n = c["h"].ptr, c["n"]
    assert L.gp_cov_build(h, th_(kind=4), n, 2, P(c["X"]), P(c["S"]), n) == -2
    assert L.gp_cov_build(h, th_(ls=math.nan), n, 2, P(c["X"]), P(c["S"]), n) == NONFINITE
    assert L.gp_cov_build(h, th_(lt=math.inf), n, 2, P(c["X"]), P(c["S"]), n) == NONFINITE
    assert L.gp_cov_build(h, th_(lr=-math.inf), n, 2, P(c["X"]), P(c["S"]), n) == NONFINITE
    assert L.gp_cov_build(h, th_(), -1, 2, P(c["X"]), P(c["S"]), n) == -3
    assert L.gp_cov_build(h, th_(), n, 0, P(c["X"]), P(c["S"]), n) == -4
    assert L.gp_cov_build(h, th_(), n, 17, P(c["X"]), P(c["S"]), n) == -4
    assert L.gp_cov_build(h, th_(), n, 2, None, P(c["S"]), n) == -5
    assert L.gp_cov_build(h, th_(), n, 2, P(c["X"]), None, n) == -6
    assert L.gp_cov_build(h, th_(), n, 2, P(c["X"]), P(c["S"]), n - 1) == -7
    # a log variance of -inf is an exact zero, not an error
    assert L.gp_cov_build(h, th_(ls=-math.inf, lt=-math.inf), n, 2, P(c["X"]), P(c["S"]), n) == 0


def test_potrf_and_solve_arguments(ctx):
    L, c = gp.lib(), ctx
    h, n, ws = c["h"].ptr, c["n"], c["ws"]
    A, info = P(c["S"]), P(c["info"])
    assert L.gp_potrf(h, 3, n, A, n, info, P(ws), ws.numel()) == -2
    assert L.gp_potrf(h, 0, -5, A, n, info, P(ws), ws.numel()) == -3
    assert L.gp_potrf(h, 0, n, None, n, info, P(ws), ws.numel()) == -4
    assert L.gp_potrf(h, 0, n, A, n - 1, info, P(ws), ws.numel()) == -5
    assert L.gp_potrf(h, 0, n, A, n, None, P(ws), ws.numel()) == -6
    assert L.gp_potrf(h, 0, n, A, n, info, None, ws.numel()) == -7
    assert L.gp_potrf(h, 0, n, A, n, info, P(ws), 16) == WS_TOO_SMALL
    x = P(c["y"])
    assert L.gp_trsv(h, 2, n, A, n, x, P(ws), ws.numel()) == -2
    assert L.gp_trsv(h, 0, n, A, 0, x, P(ws), ws.numel()) == -5
    assert L.gp_trsv(h, 0, n, A, n, None, P(ws), ws.numel()) == -6
    assert L.gp_trsv(h, 0, n, A, n, x, P(ws), 8) == WS_TOO_SMALL
    assert L.gp_trsm(h, 0, n, -1, A, n, x, n, P(ws), ws.numel()) == -4
    assert L.gp_trsm(h, 0, n, 1, A, n, x, n - 1, P(ws), ws.numel()) == -8
    torch.cuda.synchronize()
    assert int(c["info"].item()) == 5, "a rejected call must enqueue nothing"


def test_loglik_arguments(ctx):
    L, c = gp.lib(), ctx
    h, n, ws = c["h"].ptr, c["n"], c["ws"]
    X, y, S, o, g, i = P(c["X"]), P(c["y"]), P(c["S"]), P(c["out3"]), P(c["grad"]), P(c["info"])
    W, nb = P(ws), ws.numel()
    assert L.gp_loglik(h, th_(ls=math.nan), 0, n, 2, X, y, None, S, n, o, None, i, None, W, nb) == NONFINITE
    assert L.gp_loglik(h, th_(), 7, n, 2, X, y, None, S, n, o, None, i, None, W, nb) == -3
    assert L.gp_loglik(h, th_(), 0, -1, 2, X, y, None, S, n, o, None, i, None, W, nb) == -4
    assert L.gp_loglik(h, th_(), 0, n, 2, X, None, None, S, n, o, None, i, None, W, nb) == -7
    assert L.gp_loglik(h, th_(), 0, n, 2, X, y, None, S, n - 3, o, None, i, None, W, nb) == -10
    assert L.gp_loglik(h, th_(), 0, n, 2, X, y, None, S, n, None, None, i, None, W, nb) == -11
    assert L.gp_loglik(h, th_(), 0, n, 2, X, y, None, S, n, o, None, None, None, W, nb) == -13
    assert L.gp_loglik(h, th_(), 0, n, 2, X, y, None, S, n, o, None, i, None, None, nb) == -15
    assert L.gp_loglik(h, th_(), 0, n, 2, X, y, None, S, n, o, None, i, None, W, 1024) == WS_TOO_SMALL
    assert L.gp_loglik_grad(h, th_(), 0, n, 2, X, y, None, S, n, o, None, None, i, None, W, nb) == -12
    assert L.gp_loglik_grad(h, th_(lt=math.inf), 0, n, 2, X, y, None, S, n, o, g, None, i, None, W,
                            nb) == NONFINITE
    torch.cuda.synchronize()
    assert np.all(c["out3"].cpu().numpy() == 7.0) and int(c["info"].item()) == 5


def test_krige_batched_and_options_arguments(ctx):
    L, c = gp.lib(), ctx
    h, n, ws = c["h"].ptr, c["n"], c["ws"]
    X, S = P(c["X"]), P(c["S"])
    kws = c["h"].workspace(gp.GP_OP_KRIGE, n, 10)
    mean = torch.empty(10, dtype=torch.float64, device="cuda")
    var = torch.empty(10, dtype=torch.float64, device="cuda")
    args = lambda **kw: [h, th_(), n, 10, 2, X, X, S, kw.get("ldl", n), P(c["y"]), kw.get("mu", 0.0),  # noqa: E731
                         P(mean), P(var), 0, P(kws), kw.get("wsb", kws.numel())]
    assert L.gp_krige(*args(mu=math.nan)) == NONFINITE
    assert L.gp_krige(*args(mu=math.inf)) == NONFINITE
    assert L.gp_krige(*args(ldl=n - 1)) == -9
    assert L.gp_krige(*args(wsb=256)) == WS_TOO_SMALL
    o = gp.Options()
    assert L.gp_get_options(h, ctypes.byref(o)) == 0
    bad = gp.Options.from_buffer_copy(o)
    bad.ir_tol = math.nan
    assert L.gp_set_options(h, ctypes.byref(bad)) == NONFINITE
    bad = gp.Options.from_buffer_copy(o)
    bad.nb = 100
    assert L.gp_set_options(h, ctypes.byref(bad)) == -2
    bad = gp.Options.from_buffer_copy(o)
    bad.fail_inject = 4
    assert L.gp_set_options(h, ctypes.byref(bad)) == -2
    b = ctypes.c_size_t()
    assert L.gp_workspace_size(h, 99, n, 0, 0, ctypes.byref(b)) == -2
    assert L.gp_workspace_size(h, gp.GP_OP_LOGLIK, -1, 0, 0, ctypes.byref(b)) == -3
    sizes = np.array([100, -1], dtype=np.int64)
    offs = np.zeros(2, dtype=np.int64)
    ths = (gp.Theta * 2)(th_(), th_())
    out3 = torch.empty(6, dtype=torch.float64, device="cuda")
    info = torch.empty(2, dtype=torch.int32, device="cuda")
    rc = L.gp_loglik_batched(h, 2, ctypes.cast(ths, ctypes.c_void_p), sizes.ctypes.data_as(ctypes.c_void_p),
                             offs.ctypes.data_as(ctypes.c_void_p), offs.ctypes.data_as(ctypes.c_void_p), 2, X,
                             P(c["y"]), S, P(out3), P(info), P(ws), ws.numel())
    assert rc == -4
    ths[1].log_rho = math.nan
    sizes[1] = 10
    rc = L.gp_loglik_batched(h, 2, ctypes.cast(ths, ctypes.c_void_p), sizes.ctypes.data_as(ctypes.c_void_p),
                             offs.ctypes.data_as(ctypes.c_void_p), offs.ctypes.data_as(ctypes.c_void_p), 2, X,
                             P(c["y"]), S, P(out3), P(info), P(ws), ws.numel())
    assert rc == NONFINITE
    assert L.gp_loglik_batched(h, -1, None, None, None, None, 2, X, P(c["y"]), S, P(out3), P(info), P(ws),
                               ws.numel()) == -2
