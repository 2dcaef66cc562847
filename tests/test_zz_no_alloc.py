"""gp_loglik_noalloc (static per-device workspace) against gp_loglik.

Two calls in a row through the C ABI, the second with a smaller problem (so
the static array holds the first call's larger contents when the second
starts), each compared with gp_loglik on the same inputs and a caller-owned
workspace: loglik, log|C|, q at 1e-11 relative (the FP64 bar), the factor
element-wise and alpha.  Then a mixed-precision call, the size limit and the
argument checks.
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

SCRATCH_BYTES = 128 << 20  # GP_SCRATCH_BYTES of include/gpmi.h


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


def data(n, seed, kernel=1, rho=0.05, t2=0.01):
    X = synth.uniform_points(n, seed)
    y = synth.smooth_field(X, seed + 100, ell=rho, t2=t2)
    th = gp.theta(kernel, log=[0.0, math.log(rho), math.log(t2)])
    return torch.as_tensor(X, device="cuda"), torch.as_tensor(y, device="cuda"), th


def compare(r0, r1, n, tol=1e-11):
    assert int(r0["info"].item()) == 0 and int(r1["info"].item()) == 0
    a, b = r0["out3"].cpu().numpy(), r1["out3"].cpu().numpy()
    rel = np.abs(a - b) / np.abs(a)
    L0 = torch.tril(r0["S"][:n, :n].T)
    L1 = torch.tril(r1["S"][:n, :n].T)
    dl = (L0 - L1).abs().max().item() / L0.diagonal().abs().max().item()
    da = ((r0["alpha"] - r1["alpha"]).norm() / r0["alpha"].norm()).item()
    print("n=%d: rel diff loglik %.2e logdet %.2e q %.2e; factor %.2e; alpha %.2e" % (n, *rel, dl, da))
    assert np.all(rel <= tol), rel
    assert dl <= 1e-12 and da <= 1e-10


def test_two_calls_second_smaller():
    h = gp.handle()
    ws_need = ctypes.c_size_t()
    gp.check(gp.lib().gp_workspace_size(h.ptr, gp.GP_OP_LOGLIK, 9000, 0, gp.GP_FP64, ctypes.byref(ws_need)))
    assert ws_need.value <= SCRATCH_BYTES
    for n, seed in ((9000, 7), (2500, 8)):  # several 768-column panels, then fewer; ragged tails
        X, y, th = data(n, seed)
        r_ref = gp.loglik(X, y, th, want_alpha=True)
        r_na = gp.loglik_noalloc(X, y, th, want_alpha=True)
        torch.cuda.synchronize()
        compare(r_ref, r_na, n)


def test_mixed_fp32_and_repeat():
    # the mixed path uses more of the array (Morton keys, permuted points,
    # residual partials); a repeated call must give the same numbers
    X, y, th = data(4000, 11, kernel=0, rho=0.1, t2=0.1)
    r_ref = gp.loglik(X, y, th, prec=gp.GP_FP32_TRAIL, want_alpha=True)
    r1 = gp.loglik_noalloc(X, y, th, prec=gp.GP_FP32_TRAIL, want_alpha=True)
    o1 = r1["out3"].cpu().numpy()
    a = r_ref["out3"].cpu().numpy()
    assert np.all(np.abs(o1 - a) <= 1e-11 * np.abs(a)), (o1, a)
    X2, y2, th2 = data(1000, 12, kernel=0, rho=0.1, t2=0.1)
    r2 = gp.loglik_noalloc(X2, y2, th2, prec=gp.GP_FP32_TRAIL, want_alpha=True)
    r2_ref = gp.loglik(X2, y2, th2, prec=gp.GP_FP32_TRAIL, want_alpha=True)
    o2, a2 = r2["out3"].cpu().numpy(), r2_ref["out3"].cpu().numpy()
    assert np.all(np.abs(o2 - a2) <= 1e-11 * np.abs(a2)), (o2, a2)
    assert r2["ir"][2].item() == 1.0


def test_size_limit_and_arguments():
    h = gp.handle()
    lib = gp.lib()
    # smallest n (multiple of 256) whose FP64 workspace exceeds the array
    n = 256
    b = ctypes.c_size_t()
    while True:
        gp.check(lib.gp_workspace_size(h.ptr, gp.GP_OP_LOGLIK, n, 0, gp.GP_FP64, ctypes.byref(b)))
        if b.value > SCRATCH_BYTES:
            break
        n += 256
    X, y, th = data(n, 3)
    S = gp.colmajor_storage(n)  # real buffers: a wrong check would compute, not fault
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = gp._ptr
    rc = lib.gp_loglik_noalloc(h.ptr, th, gp.GP_FP64, n, 2, p(X), p(y), None, p(S), S.shape[1], p(out3), None,
                               p(info), None)
    print("n=%d needs %d bytes: rc %d (%s)" % (n, b.value, rc, lib.gp_strerror(rc).decode()))
    assert rc == -1006
    del S
    torch.cuda.empty_cache()
    X, y, th = data(100, 4)
    S = gp.colmajor_storage(100)
    args = [h.ptr, th, gp.GP_FP64, 100, 2, p(X), p(y), None, p(S), S.shape[1], p(out3), None, p(info), None]
    assert lib.gp_loglik_noalloc(None, *args[1:]) == -1
    bad = list(args)
    bad[9] = 50  # ldc < n
    assert lib.gp_loglik_noalloc(*bad) == -10
    bad = list(args)
    bad[10] = None  # out3
    assert lib.gp_loglik_noalloc(*bad) == -11
    bad = list(args)
    bad[1] = gp.theta(0, log=[float("nan"), 0.0, 0.0])
    assert lib.gp_loglik_noalloc(*bad) == -1001
