"""GPU parity of the many-right-hand-side triangular solve, kriging (mean and
variance, Section 1's prediction and its uncertainty) and the adjoint
gradient of the log-likelihood (Rasmussen & Williams 2006, eq. 5.9) against
the CPU oracle, plus central finite differences of the GPU log-likelihood.

Tolerances: solve normwise 1e-12; kriging mean 1e-10 relative, variance
1e-10 sigma^2 absolute (it cancels); gradient 1e-9 normwise relative to the
oracle and 1e-6 max(1, |g|) against central differences with h = 1e-5.
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
    return np.array([math.log(s2), math.log(rho), math.log(t2)])


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,nrhs", [(1, 3), (64, 5), (300, 130), (1000, 257)])
@pytest.mark.parametrize("trans", [False, True])
def test_trsm_parity(orc, n, nrhs, trans):
    X = synth.uniform_points(n, 300 + n)
    Lo, _ = orc.potrf(orc.cov(1, logth(1.0, 0.1, 0.05), X))
    rng = np.random.default_rng(5)
    Bm = rng.standard_normal((n, nrhs))
    S = gp.colmajor_storage(n, ld=n + 2)
    gp.colmajor(S, n).copy_(torch.as_tensor(Lo))
    Bs = gp.colmajor_storage(n, nrhs, ld=n + 1)
    gp.colmajor(Bs, n).copy_(torch.as_tensor(Bm))
    gp.trsm(S, n, Bs, trans=trans)
    got = gp.colmajor(Bs, n).cpu().numpy()
    ref = np.stack([orc.trsv(Lo, Bm[:, j], trans=trans) for j in range(nrhs)], axis=1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12


@pytest.mark.parametrize("n,m,kernel,nug", [(1, 4, 0, False), (200, 70, 1, False), (1500, 513, 1, True),
                                            (3000, 256, 2, False)])
def test_krige_parity(orc, n, m, kernel, nug):
    X = synth.uniform_points(n, 400 + n)
    Xs = synth.uniform_points(m, 401 + n)
    y = synth.smooth_field(X, 402, ell=0.05, t2=0.01)
    t = logth(1.0, 0.05, 0.01)
    mu = 0.2
    (_, _, _), Lo, alpha_o = orc.loglik(kernel, t, X, y, mu=mu, want=True)
    mean_o, var_o = orc.krige(kernel, t, X, Xs, Lo, alpha_o, mu=mu, include_nugget=nug)
    r = gp.loglik(dev(X), dev(y), gp.theta(kernel, log=t), mu=mu, want_alpha=True)
    mean, var = gp.krige(dev(X), dev(Xs), r["S"], r["alpha"], gp.theta(kernel, log=t), mu=mu, include_nugget=nug)
    mean, var = mean.cpu().numpy(), var.cpu().numpy()
    assert np.max(np.abs(mean - mean_o)) <= 1e-10 * max(1.0, np.max(np.abs(mean_o)))
    assert np.max(np.abs(var - var_o)) <= 1e-10


def test_krige_compound_symmetry_closed_form():
    n, m = 4096, 33
    X = synth.uniform_points(n, 9)
    y = synth.normals(n, 10) + 0.3
    s2, t2 = 0.8, 0.45
    th = gp.theta(0, s2, 1e300, t2)
    r = gp.loglik(dev(X), dev(y), th, want_alpha=True)
    mean, var = gp.krige(dev(X), dev(synth.uniform_points(m, 99)), r["S"], r["alpha"], th)
    den = t2 + n * s2
    np.testing.assert_allclose(mean.cpu().numpy(), s2 * y.sum() / den, rtol=1e-9)
    np.testing.assert_allclose(var.cpu().numpy(), s2 * t2 / den, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("n,kernel", [(1, 0), (64, 1), (129, 2), (700, 1), (1500, 0), (2100, 2)])
def test_grad_parity(orc, n, kernel):
    X = synth.uniform_points(n, 500 + n)
    y = synth.smooth_field(X, 501, ell=0.08, t2=0.02)
    t = logth(0.9, 0.08, 0.02)
    (ll_o, _, _), g_o = orc.loglik_grad(kernel, t, X, y)
    r = gp.loglik_grad(dev(X), dev(y), gp.theta(kernel, log=t))
    out = r["out3"].cpu().numpy()
    g = r["grad"].cpu().numpy()
    assert int(r["info"].item()) == 0
    assert abs(out[0] - ll_o) <= 1e-11 * abs(ll_o)
    assert np.linalg.norm(g - g_o) <= 1e-9 * max(1.0, np.linalg.norm(g_o)), (g, g_o)


def test_grad_central_fd_and_scale_identity():
    n = 2048
    X = synth.uniform_points(n, 600)
    y = synth.smooth_field(X, 601, ell=0.05, t2=0.01)
    t = logth(1.0, 0.05, 0.01)
    r = gp.loglik_grad(dev(X), dev(y), gp.theta(1, log=t))
    g = r["grad"].cpu().numpy()
    ll, ld, q = r["out3"].cpu().numpy()
    assert abs((g[0] + g[2]) - 0.5 * (q - n)) <= 1e-8 * max(1.0, abs(q))
    h = 1e-5
    for k in range(3):
        tp, tm = t.copy(), t.copy()
        tp[k] += h
        tm[k] -= h
        fp = gp.loglik(dev(X), dev(y), gp.theta(1, log=tp))["out3"][0].item()
        fm = gp.loglik(dev(X), dev(y), gp.theta(1, log=tm))["out3"][0].item()
        fd = (fp - fm) / (2 * h)
        assert abs(g[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)


def test_autograd_function_matches_oracle_gradient(orc):
    """log_likelihood is a torch.autograd.Function: its backward is the adjoint."""
    n = 500
    X = synth.uniform_points(n, 650)
    y = synth.smooth_field(X, 651, ell=0.1, t2=0.05)
    t = logth(1.3, 0.1, 0.05)
    (ll_o, _, _), g_o = orc.loglik_grad(2, t, X, y)
    lt = torch.tensor(t, dtype=torch.float64, requires_grad=True)
    ll = gp.log_likelihood(dev(X), dev(y), lt, kernel="matern52")
    ll.backward()
    assert abs(ll.item() - ll_o) <= 1e-11 * abs(ll_o)
    g = lt.grad.numpy()
    assert np.linalg.norm(g - g_o) <= 1e-9 * max(1.0, np.linalg.norm(g_o)), (g, g_o)
    # chain rule through a function of log_theta
    lt2 = torch.tensor(t, dtype=torch.float64, requires_grad=True)
    (3.0 * gp.log_likelihood(dev(X), dev(y), lt2, kernel=2)).backward()
    assert np.linalg.norm(lt2.grad.numpy() - 3.0 * g_o) <= 3e-9 * max(1.0, np.linalg.norm(g_o))
    # no gradient requested: plain evaluation
    with torch.no_grad():
        v = gp.log_likelihood(dev(X), dev(y), torch.tensor(t, dtype=torch.float64), kernel=2)
    assert abs(v.item() - ll_o) <= 1e-11 * abs(ll_o)


def test_autograd_not_pd_raises():
    X = np.zeros((5, 2))
    y = np.ones(5)
    lt = torch.tensor([0.0, math.log(0.1), -math.inf], dtype=torch.float64, requires_grad=True)
    with pytest.raises(gp.NotPositiveDefinite):
        gp.log_likelihood(dev(X), dev(y), lt)
