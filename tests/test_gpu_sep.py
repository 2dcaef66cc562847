"""GPU parity for the spectral example's covariance family (Section 4.2):
a product of smoothness-2 Matern correlations in phase and log-wavelength,
a random effect shared by the observations of one phase and known
per-observation noise variances.  Points are (t, w, v) rows on a phase x
wavelength grid (the layout of the paper's data), parameters the paper's
estimates (sigma^2 = 0.0071, rho_t = 2.33, tau^2 = 2.6e-5, rho_w = 0.0089).

Tolerances.  Covariance entries: 2e-14 relative (both sides evaluate K_2
to a few ulp by different methods: the GPU by series / quadrature /
asymptotic expansion by range, the oracle by one quadrature).  Log-
likelihood, log|C|, q: 1e-11 relative (the FP64 bar).  Gradient: 1e-9
normwise against the oracle, central differences (h = 1e-5) to
1e-6 max(1, |g_k|).  Kriging mean 1e-10 relative (floor: the field's sd),
variance 1e-10 sigma^2 absolute.
"""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1305_4886_amd as gp  # noqa: E402
from paper_1305_4886_amd import synth  # noqa: E402

EST = (0.0071, 2.33, 2.6e-5, 0.0089)
LOG_EST = np.log(np.array(EST))


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def th_of(lt):
    return gp.theta(gp.GP_SEP_MATERN2, log=lt)


def data(n_phase, n_wave, seed, lt=LOG_EST):
    X = synth.spectral_points(n_phase, n_wave, seed)
    C = oracle.cov(3, lt, X)
    L, info = oracle.potrf(C)
    assert info == 0
    y = L @ synth.normals(X.shape[0], seed + 1)
    return X, y


def test_matern2_across_its_regimes():
    # pairs at phase distance r rho_t (same wavelength, no random effect):
    # C_{2k+1, 2k} = sigma^2 M(r)
    rs = np.array([1e-12, 1e-6, 0.01, 0.3, 1.0, 1.999, 2.0, 2.001, 3.0, 7.5, 12.0, 19.99, 20.0, 20.01, 35.0,
                   80.0, 300.0, 650.0])
    s2, rt = 1.3, 1.7
    X = np.zeros((2 * len(rs), 3))
    X[1::2, 0] = rs * rt
    X[0::2, 0] = 0.0
    X[:, 0] += np.repeat(np.arange(len(rs)) * 1e4, 2)  # pairs far apart from each other
    lt = np.array([math.log(s2), math.log(rt), math.log(0.5), math.log(0.1)])
    S = gp.cov_build(dev(X), th_of(lt))
    got = np.array([S[2 * k, 2 * k + 1].item() for k in range(len(rs))])  # storage [j, i] = C(i, j)
    ref = np.array([oracle.cov(3, lt, X[2 * k:2 * k + 2])[1, 0] for k in range(len(rs))])
    rel = np.abs(got - ref) / ref
    print("M(r) rel err by r:", dict(zip(rs.tolist(), rel.tolist())))
    assert rel.max() <= 2e-14


@pytest.mark.parametrize("n_phase,n_wave", [(3, 50), (4, 257)])
def test_sep_cov_build_parity(n_phase, n_wave):
    X = synth.spectral_points(n_phase, n_wave, 3)
    n = X.shape[0]
    S = gp.cov_build(dev(X), th_of(LOG_EST))
    got = np.tril(S[:n, :n].T.cpu().numpy())
    ref = np.tril(oracle.cov(3, LOG_EST, X))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("n=%d: max |dC| / max |C| = %.2e" % (n, err))
    assert np.all(np.abs(got - ref) <= 2e-14 * np.abs(ref) + 1e-30)
    Xs = X[::7].copy()
    Xs[:, 2] = 0.0
    Cs = gp.cross_cov_build(dev(X), dev(Xs), th_of(LOG_EST))
    gcs = Cs[:Xs.shape[0], :n].T.cpu().numpy()
    rcs = oracle.cross_cov(3, LOG_EST, X, Xs)
    assert np.all(np.abs(gcs - rcs) <= 2e-14 * np.abs(rcs) + 1e-30)


@pytest.mark.parametrize("n_phase,n_wave", [(5, 300), (3, 700)])
def test_sep_loglik_gradient_parity(n_phase, n_wave):
    X, y = data(n_phase, n_wave, 20 + n_wave)
    n = X.shape[0]
    r = gp.loglik(dev(X), dev(y), th_of(LOG_EST), want_alpha=True)
    assert int(r["info"].item()) == 0
    (ll, ld, q), L, a = oracle.loglik(3, LOG_EST, X, y, want=True)
    out = r["out3"].cpu().numpy()
    e = np.abs(out - np.array([ll, ld, q])) / np.abs([ll, ld, q])
    ea = np.linalg.norm(r["alpha"].cpu().numpy() - a) / np.linalg.norm(a)
    print("n=%d: rel err loglik %.2e logdet %.2e q %.2e alpha %.2e" % (n, *e, ea))
    assert np.all(e <= 1e-11)
    assert ea <= 1e-8
    rg = gp.loglik_grad(dev(X), dev(y), th_of(LOG_EST))
    g = rg["grad"].cpu().numpy()
    (_, _, _), gref = oracle.loglik_grad(3, LOG_EST, X, y)
    eg = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print("gradient %s oracle %s rel %.2e" % (g, gref, eg))
    assert g.shape == (4,) and eg <= 1e-9
    if n <= 1500:
        h = 1e-5
        for k in range(4):
            tp, tm = LOG_EST.copy(), LOG_EST.copy()
            tp[k] += h
            tm[k] -= h
            fd = (gp.loglik(dev(X), dev(y), th_of(tp))["out3"][0].item() -
                  gp.loglik(dev(X), dev(y), th_of(tm))["out3"][0].item()) / (2 * h)
            assert abs(g[k] - fd) <= 1e-6 * max(1.0, abs(g[k])), (k, g[k], fd)


def test_sep_kriging_parity():
    X, y = data(4, 400, 41)
    r = gp.loglik(dev(X), dev(y), th_of(LOG_EST), want_alpha=True)
    # a dense wavelength line at an observed phase and at a phase between nights
    w = np.linspace(X[0, 1], X[399, 1], 300)
    t_new = np.concatenate([np.full(150, X[400, 0]), np.full(150, 0.5 * (X[0, 0] + X[400, 0]))])
    Xs = np.column_stack([t_new, np.concatenate([w[:150], w[150:]]), np.zeros(300)])
    mean, var = gp.krige(dev(X), dev(Xs), r["S"], r["alpha"], th_of(LOG_EST))
    (_, _, _), L, a = oracle.loglik(3, LOG_EST, X, y, want=True)
    mref, vref = oracle.krige(3, LOG_EST, X, Xs, L, a)
    em = np.abs(mean.cpu().numpy() - mref).max()
    ev = np.abs(var.cpu().numpy() - vref).max()
    print("kriging: max |d mean| %.2e (sd %.2e), max |d var| %.2e" % (em, math.sqrt(EST[0]), ev))
    assert em <= 1e-10 * math.sqrt(EST[0])
    assert ev <= 1e-10 * EST[0]


def test_sep_argument_checks():
    lib = gp.lib()
    h = gp.handle()
    X = dev(synth.spectral_points(2, 10, 1))
    S = gp.colmajor_storage(20)
    p = gp._ptr
    th = th_of(LOG_EST)
    assert lib.gp_cov_build(h.ptr, th, 20, 2, p(X), p(S), 20) == -4  # the family needs (t, w, v)
    bad = th_of(LOG_EST)
    bad.log_rho2 = float("nan")
    assert lib.gp_cov_build(h.ptr, bad, 20, 3, p(X), p(S), 20) == -1001
    sizes = np.array([20], dtype=np.int64)
    with pytest.raises(gp.GPError) as ei:
        gp.loglik_batched(X, dev(np.zeros(20)), [th], sizes)
    assert ei.value.code == -1004
