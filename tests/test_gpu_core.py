"""GPU parity of the covariance build, blocked Cholesky, triangular solves and
log-likelihood against the CPU oracle (Section 1 of the paper: build C(theta),
L L^T = C, L^{-1}(y - mu), log-determinant, marginal log-likelihood).

Tolerances: the FP64 path computes the same mathematical objects in another
summation order, so differences are at rounding level amplified by the
conditioning of C.  Covariance entries: 1e-14 relative (device exp/sqrt vs
libm, a few ulp).  Factor: normwise 1e-12.  Log-likelihood: 1e-11 relative.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1305_4886_amd as gp  # noqa: E402
from paper_1305_4886_amd import synth  # noqa: E402


def logth(s2, rho, t2):
    return np.array([math.log(s2) if s2 > 0 else -np.inf, math.log(rho), math.log(t2) if t2 > 0 else -np.inf])


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def lower_of(S, n):
    return np.tril(gp.colmajor(S, n).cpu().numpy())


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,kernel,dim", [(1, 0, 2), (3, 1, 2), (65, 2, 2), (200, 0, 3), (1000, 1, 2), (1031, 2, 1)])
def test_cov_build(orc, n, kernel, dim):
    X = synth.uniform_points(n, 7, dim=dim)
    t = logth(1.3, 0.11, 0.07)
    ld = n + 5
    S = gp.colmajor_storage(n, ld=ld)
    S.fill_(7.5)
    gp.cov_build(dev(X), gp.theta(kernel, log=t), S)
    M = gp.colmajor(S, n).cpu().numpy()
    ref = orc.cov(kernel, t, X)
    il = np.tril_indices(n)
    np.testing.assert_allclose(M[il], ref[il], rtol=1e-14, atol=1e-300)
    iu = np.triu_indices(n, 1)
    assert np.all(M[iu] == 7.5), "upper triangle must stay untouched"
    assert np.all(S[:, n:].cpu().numpy() == 7.5), "padding rows beyond n untouched"


@pytest.mark.parametrize("n,m", [(1, 1), (70, 130), (1000, 257)])
def test_cross_cov(orc, n, m):
    X = synth.uniform_points(n, 8)
    Xs = synth.uniform_points(m, 9)
    t = logth(0.9, 0.2, 0.3)
    S = gp.cross_cov_build(dev(X), dev(Xs), gp.theta(1, log=t))
    M = gp.colmajor(S, n).cpu().numpy()
    np.testing.assert_allclose(M, orc.cross_cov(1, t, X, Xs), rtol=1e-14, atol=1e-300)


# (n, panel width (0: the default), lookahead, compute units reserved for the
#  lookahead chain, fused panel kernel or the per-64-column launch chain,
#  leading dimension - n, tail panel width (-1: none, 0: the default)).  An odd
#  leading dimension keeps the trailing update on its 4-byte copies; an even
#  one (ld = n with even n, the benchmark's layout, or ld = n + 1 or n + 3
#  with odd n, where the last row pair of a ragged tile reads the element past
#  the matrix) takes the 16-byte copies of the main trailing-update kernel.
#  A tail width w takes over once at most 24 w columns remain.
POTRF_CASES = [
    (1, 256, 1, 8, 1, 3, -1), (2, 256, 1, 8, 1, 3, -1), (63, 256, 1, 8, 1, 3, -1), (64, 256, 1, 8, 1, 3, -1),
    (65, 256, 1, 8, 1, 3, -1), (127, 64, 0, 0, 1, 3, -1), (200, 128, 1, 8, 1, 3, -1), (257, 256, 1, 0, 1, 3, -1),
    (500, 64, 1, 8, 1, 3, -1), (1000, 256, 1, 8, 1, 3, -1), (1000, 256, 0, 8, 1, 3, -1),
    (1100, 128, 1, 0, 1, 3, -1), (2048, 512, 1, 8, 1, 3, -1), (3001, 256, 1, 16, 1, 3, -1),
    (3001, 192, 1, 8, 1, 3, -1), (4500, 512, 1, 8, 1, 3, -1), (3001, 768, 1, 0, 1, 3, -1),
    (2500, 1024, 1, 0, 1, 3, -1), (2500, 1024, 0, 0, 1, 3, -1),
    (127, 64, 0, 0, 0, 3, -1), (1000, 256, 1, 8, 0, 3, -1), (3001, 192, 1, 8, 0, 3, -1), (4500, 512, 1, 0, 0, 3, -1),
    # the benchmark's configuration: default panel width, lookahead, ld = n
    (8192, 0, 1, 0, 1, 0, 0), (4096, 0, 1, 0, 1, 0, 0), (3000, 0, 1, 0, 1, 0, 0), (4000, 512, 0, 0, 1, 0, 0),
    (2050, 0, 1, 0, 1, 2, 0),
    # wide panels, then narrow ones for the last columns (both trailing-update copy widths,
    # with and without lookahead, reserved compute units, the launch-chain panels)
    (4500, 512, 1, 0, 1, 0, 128), (4500, 512, 1, 8, 1, 3, 128), (4500, 512, 0, 0, 1, 0, 128),
    (8192, 768, 1, 0, 1, 0, 256), (3001, 384, 1, 0, 0, 3, 64), (700, 768, 1, 0, 1, 0, 0),
    (2500, 1024, 1, 0, 1, 0, 0),
    # split lookahead updates (16-byte copies, ld = n) with compute units reserved
    # for the panel chain, and with a panel width that is not a multiple of 128
    (4096, 512, 1, 8, 1, 0, -1), (4098, 576, 1, 0, 1, 0, -1),
    # odd n with an even leading dimension (16-byte copies over an odd row count):
    # default panel width with split updates, wide then narrow panels, no
    # lookahead, the launch-chain panels with reserved compute units
    (4097, 0, 1, 0, 1, 1, 0), (3001, 512, 1, 0, 1, 1, 128), (2049, 256, 0, 0, 1, 1, -1),
    (1001, 256, 1, 8, 0, 1, -1), (8191, 768, 1, 0, 1, 1, 0),
]


@pytest.mark.parametrize("n,nb,la,pc,fused,pad,tail", POTRF_CASES)
def test_potrf_parity(orc, n, nb, la, pc, fused, pad, tail):
    X = synth.uniform_points(n, 100 + n)
    t = logth(1.0, 0.1, 0.1)
    C = orc.cov(0, t, X)
    S = gp.colmajor_storage(n, ld=n + pad)
    S.fill_(-3.25)
    gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(C) + np.triu(np.full((n, n), -3.25), 1)))
    del C
    h = gp.handle()
    saved = h.options()
    h.set_options(nb=nb, lookahead=la, panel_cus=pc, fused_panel=fused, tail_nb=tail)
    try:
        plan = h.potrf_plan(n)
        print("plan (nb, panel_cus, slab, tail):", plan, flush=True)
        if tail > 0:
            assert plan[3] == min(tail, plan[0])
        info = gp.potrf(S, n)
        torch.cuda.synchronize()
    finally:
        h.set_options(nb=saved.nb, lookahead=saved.lookahead, panel_cus=saved.panel_cus,
                      fused_panel=saved.fused_panel, tail_nb=saved.tail_nb)
    assert int(info.item()) == 0
    M = gp.colmajor(S, n).cpu().numpy()
    assert np.all(M[np.triu_indices(n, 1)] == -3.25), "upper triangle must stay untouched"
    L = np.tril(M)
    del M
    C = orc.cov(0, t, X)
    Lo, info_o = orc.potrf(C)
    assert info_o == 0
    err = np.linalg.norm(L - Lo) / np.linalg.norm(Lo)
    assert err <= 1e-12, err
    rec = np.linalg.norm(L @ L.T - C) / np.linalg.norm(C)
    assert rec <= 20 * n * np.finfo(float).eps


@pytest.mark.parametrize("bad", [0, 63, 64, 130, 700])
def test_potrf_not_pd_reports_column(orc, bad):
    n = 900
    A = np.eye(n) * 2.0 + 0.01
    A[bad, bad] = -1.0
    S = gp.colmajor_storage(n)
    gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(A)))
    info = gp.potrf(S, n)
    _, info_o = orc.potrf(A)
    assert int(info.item()) == info_o == bad + 1


@pytest.mark.parametrize("n", [1, 64, 65, 128, 129, 192, 256, 333, 1000, 2500])
@pytest.mark.parametrize("trans", [False, True])
def test_trsv_parity(orc, n, trans):
    X = synth.uniform_points(n, 200 + n)
    t = logth(1.0, 0.15, 0.05)
    C = orc.cov(2, t, X)
    Lo, _ = orc.potrf(C)
    b = synth.normals(n, 201)
    S = gp.colmajor_storage(n, ld=n + 1)
    gp.colmajor(S, n).copy_(torch.as_tensor(Lo))
    x = dev(b.copy())
    gp.trsv(S, n, x, trans=trans)
    ref = orc.trsv(Lo, b, trans=trans)
    got = x.cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12


def test_loglik_workload_exp_n1024(orc):
    """n = 1024 uniform points, exponential sigma^2 = 1, rho = 0.1, tau^2 = 0.1,
    y = L z drawn with the oracle's Cholesky (seeded)."""
    w = synth.WORKLOADS["exp_n1024"]
    X = synth.uniform_points(w["n"], w["seed"])
    t = logth(w["sigma2"], w["rho"], w["tau2"])
    Lo, _ = orc.potrf(orc.cov(0, t, X))
    y = Lo @ synth.normals(w["n"], w["seed"] + 1000)
    (ll, ld, q), _, alpha_o = orc.loglik(0, t, X, y, want=True)
    r = gp.loglik(dev(X), dev(y), gp.theta(0, log=t), want_alpha=True)
    out = r["out3"].cpu().numpy()
    assert int(r["info"].item()) == 0
    assert abs(out[0] - ll) <= 1e-11 * abs(ll), (out, ll)
    assert abs(out[1] - ld) <= 1e-11 * abs(ld)
    assert abs(out[2] - q) <= 1e-11 * abs(q)
    a = r["alpha"].cpu().numpy()
    assert np.linalg.norm(a - alpha_o) / np.linalg.norm(alpha_o) <= 1e-10


@pytest.mark.parametrize("n,kernel,seed", [(1, 0, 1), (100, 1, 2), (777, 2, 3), (2049, 1, 4)])
def test_loglik_parity_mu(orc, n, kernel, seed):
    X = synth.uniform_points(n, seed)
    y = synth.smooth_field(X, seed + 1, ell=0.1, t2=0.02)
    mu = np.linspace(-0.5, 0.5, n)
    t = logth(0.8, 0.07, 0.02)
    ll, ld, q = orc.loglik(kernel, t, X, y, mu=mu)
    r = gp.loglik(dev(X), dev(y), gp.theta(kernel, log=t), mu=dev(mu))
    out = r["out3"].cpu().numpy()
    assert abs(out[0] - ll) <= 1e-11 * abs(ll), (out, ll)


def test_loglik_not_pd_gives_nan_and_info():
    n = 300
    X = synth.uniform_points(n, 5)
    X[200] = X[10]
    r = gp.loglik(dev(X), dev(np.ones(n)), gp.theta(0, 1.0, 0.2, 0.0))
    info = int(r["info"].item())
    out = r["out3"].cpu().numpy()
    if info:
        assert info >= 201 and np.all(np.isnan(out))
    else:  # rounding left a tiny positive pivot at the duplicate
        assert np.all(np.isfinite(out))


def test_compound_symmetry_n8192():
    """Closed form at a size that exercises many panels: C = t2 I + s2 11^T."""
    n = 8192
    X = synth.uniform_points(n, 9)
    y = synth.normals(n, 10) + 0.3
    s2, t2 = 0.8, 0.45
    r = gp.loglik(dev(X), dev(y), gp.theta(0, s2, 1e300, t2))
    ll, ld, q = r["out3"].cpu().numpy()
    den = t2 + n * s2
    ld_ref = (n - 1) * math.log(t2) + math.log(den)
    sy, yy = float(y.sum()), float(y @ y)
    q_ref = (yy - s2 * sy * sy / den) / t2
    assert abs(ld - ld_ref) <= 1e-11 * abs(ld_ref)
    assert abs(q - q_ref) <= 1e-10 * abs(q_ref)


def test_loglik_scalar_mu_is_taken_in_fp64(orc):
    """A Python float mean must reach the device as that double, not via float32."""
    n = 300
    X = synth.uniform_points(n, 31)
    y = synth.smooth_field(X, 32, ell=0.1, t2=0.05)
    t = logth(1.0, 0.1, 0.05)
    mu = 0.2  # not representable in float32
    ll_o, _, _ = orc.loglik(0, t, X, y, mu=np.full(n, mu))
    a = gp.loglik(dev(X), dev(y), gp.theta(0, log=t), mu=mu)["out3"].cpu().numpy()
    b = gp.loglik(dev(X), dev(y), gp.theta(0, log=t), mu=dev(np.full(n, mu)))["out3"].cpu().numpy()
    assert np.array_equal(a, b)
    assert abs(a[0] - ll_o) <= 1e-11 * abs(ll_o)


def test_tune_potrf_picks_a_candidate_and_factors_correctly(orc):
    h = gp.handle()
    saved = h.options()
    try:
        times = h.tune_potrf(1500, nb=(128, 256), panel_cus=(0, 8))
        o = h.options()
        assert set(times) == {(128, 0), (128, 8), (256, 0), (256, 8)}
        assert all(t > 0 for t in times.values()), times
        assert (o.nb, o.panel_cus) == min(times, key=times.get) and o.lookahead == 1
        n = 1500
        X = synth.uniform_points(n, 77)
        t = logth(1.0, 0.1, 0.1)
        C = orc.cov(0, t, X)
        S = gp.colmajor_storage(n)
        gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(C)))
        assert int(gp.potrf(S, n).item()) == 0
        Lo, _ = orc.potrf(C)
        L = lower_of(S, n)
        assert np.linalg.norm(L - Lo) <= 1e-12 * np.linalg.norm(Lo)
    finally:
        h.set_options(nb=saved.nb, lookahead=saved.lookahead, panel_cus=saved.panel_cus, syrk_slab=saved.syrk_slab)
        h.tune_reset()
