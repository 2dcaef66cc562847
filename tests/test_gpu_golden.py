"""GPU parity at the full workload sizes against stored oracle values.

The values in ``tests/golden/*.npz`` were written by
``tests/golden/make_golden.py``, which calls only the CPU oracle (plain
Cholesky-Crout, substitution, compensated sums; Section 1 of the paper) and
the seeded input generators.  The points are regenerated here from their
seeds and checked against the stored SHA-256 of their bytes; the response y
(drawn as L z from the oracle's factor) is stored.

Workloads:
* n = 16384 Matern-3/2 (sigma^2 = 1, rho = 0.05, tau^2 = 0.01): loglik,
  log|C|, q, sampled entries of L and of alpha, kriging mean and variance at
  m = 4096 points, and the gradient (also against central differences);
* n = 32768 exponential (sigma^2 = 1, rho = 0.1, tau^2 = 0.1), the benchmark
  workload in its own launch configuration (automatic panel width, which the
  shipped tuning table sets to 640 at this size, lookahead, ld = n, so the
  16-byte-copy trailing update) and at the untuned default width 768:
  loglik, log|C|, q, sampled L and alpha; the mixed FP32 / BF16 paths
  against the same values.

The sampled entries of L sit uniformly over the lower triangle and on the
edges of the 64-, 128- and 768-wide blocks, so a tile placed or decoded
wrongly (which a compound-symmetry closed form cannot see) shows up.

Tolerances.  FP64 loglik, log|C| and q: 1e-11 relative (spec bar).
Factor entries: |dL_ij| <= 1e-10 max_j L_jj.  A backward-stable Cholesky in
another summation order differs from the oracle's by about kappa(C) n u
relative in the worst case; kappa(C) is about 3e4 here (largest eigenvalue
~ n sigma^2 2 pi rho^2 c, smallest >= tau^2), so rounding-level differences
sit near 1e-12 and 1e-10 leaves an order of magnitude while any misplaced
tile moves entries by O(1e-2) or more.  alpha: 1e-9 relative over the
sample (kappa u ~ 1e-11).  Kriging mean 1e-10 relative (floor 1) and latent
variance 1e-10 absolute (sigma^2 = 1).  Gradient: 1e-9 normwise against the
oracle; against central differences with h = 1e-5 in log-theta,
1e-6 max(1, |g_k|) (truncation h^2 |l'''| plus rounding eps |l| / h).
Mixed loglik: 1e-6 relative with the refined solve at 1e-10.
"""
import hashlib
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1305_4886_amd as gp  # noqa: E402
from paper_1305_4886_amd import synth  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
POINT_SEEDS = {"matern32_n16384": (2, 41), "exp_n32768": (4, None)}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def load(name):
    d = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    n = int(d["n"])
    seed, xs_seed = POINT_SEEDS[name]
    X = synth.uniform_points(n, seed)
    assert sha(X) == str(d["x_sha256"]), "regenerated points differ from the stored ones"
    g = {k: d[k] for k in d.files}
    g["X"] = X
    if xs_seed is not None:
        Xs = synth.uniform_points(4096, xs_seed)
        assert sha(Xs) == str(d["xs_sha256"])
        g["Xs"] = Xs
    return g


@pytest.fixture(scope="module")
def c2():
    return load("matern32_n16384")


@pytest.fixture(scope="module")
def c4():
    return load("exp_n32768")


def th_of(g):
    return gp.theta(int(g["kernel"]), log=g["theta"])


def check_fp64(g, r, label):
    n = int(g["n"])
    assert int(r["info"].item()) == 0
    ll, ld, q = r["out3"].cpu().numpy()
    e = [abs(ll - g["loglik"]) / abs(g["loglik"]), abs(ld - g["logdet"]) / abs(g["logdet"]),
         abs(q - g["q"]) / abs(g["q"])]
    S = r["S"]
    I, J = torch.as_tensor(g["l_i"], device="cuda"), torch.as_tensor(g["l_j"], device="cuda")
    Lv = S[J, I].cpu().numpy()  # storage row j is column j
    diag = S.diagonal()[:n].abs().max().item()
    dl = np.abs(Lv - g["l_val"])
    a = r["alpha"].cpu().numpy()[g["a_idx"]]
    ea = np.linalg.norm(a - g["a_val"]) / np.linalg.norm(g["a_val"])
    print("%s: rel err loglik %.2e logdet %.2e q %.2e; max |dL| %.2e (%d samples); alpha %.2e" % (
        label, e[0], e[1], e[2], dl.max(), len(dl), ea))
    assert e[0] <= 1e-11 and e[1] <= 1e-11 and e[2] <= 1e-11, e
    assert dl.max() <= 1e-10 * diag, (dl.max(), int(np.argmax(dl)))
    assert ea <= 1e-9


def test_c2_loglik_factor_and_kriging(c2):
    g = c2
    n = int(g["n"])
    th = th_of(g)
    X, y = dev(g["X"]), dev(g["y"])
    r = gp.loglik(X, y, th, want_alpha=True)
    check_fp64(g, r, "n=16384 matern32")
    mean, var = gp.krige(X, dev(g["Xs"]), r["S"], r["alpha"], th)
    mean, var = mean.cpu().numpy(), var.cpu().numpy()
    em = np.abs(mean - g["krige_mean"]) / np.maximum(1.0, np.abs(g["krige_mean"]))
    ev = np.abs(var - g["krige_var"])
    print("kriging m=4096: max rel mean err %.2e, max abs var err %.2e" % (em.max(), ev.max()))
    assert em.max() <= 1e-10 and ev.max() <= 1e-10
    assert n == 16384


def test_c3_gradient_oracle_and_central_differences(c2):
    g = c2
    X, y = dev(g["X"]), dev(g["y"])
    th = g["theta"]
    k = int(g["kernel"])
    r = gp.loglik_grad(X, y, gp.theta(k, log=th))
    assert int(r["info"].item()) == 0
    grad = r["grad"].cpu().numpy()
    eg = np.linalg.norm(grad - g["grad"]) / np.linalg.norm(g["grad"])
    ll = float(r["out3"][0].item())
    assert abs(ll - g["loglik"]) <= 1e-11 * abs(g["loglik"])
    h = 1e-5
    fd = np.zeros(3)
    S = gp.colmajor_storage(int(g["n"]))
    ws = gp.handle().workspace(gp.GP_OP_LOGLIK, int(g["n"]))
    for c in range(3):
        tp, tm = th.copy(), th.copy()
        tp[c] += h
        tm[c] -= h
        lp = gp.loglik(X, y, gp.theta(k, log=tp), S=S, ws=ws)["out3"][0].item()
        lm = gp.loglik(X, y, gp.theta(k, log=tm), S=S, ws=ws)["out3"][0].item()
        fd[c] = (lp - lm) / (2 * h)
    print("gradient %s; oracle %s (rel %.2e); central differences %s" % (grad, g["grad"], eg, fd))
    assert eg <= 1e-9
    assert np.all(np.abs(grad - fd) <= 1e-6 * np.maximum(1.0, np.abs(grad))), (grad, fd)


@pytest.mark.parametrize("nb", [0, 768])
def test_c4_fp64_benchmark_configuration(c4, nb):
    g = c4
    h = gp.handle()
    o = h.options()
    assert o.nb == 0 and o.lookahead == 1 and o.fused_panel == 1  # the defaults the benchmark runs
    try:
        h.set_options(nb=nb)
        print("panel width used:", h.potrf_plan(int(g["n"]))[0])
        r = gp.loglik(dev(g["X"]), dev(g["y"]), th_of(g), want_alpha=True)
    finally:
        h.set_options(nb=0)
    assert r["S"].shape[1] == int(g["n"])  # ld = n
    check_fp64(g, r, "n=32768 exp nb=%d" % nb)


@pytest.mark.parametrize("prec", [gp.GP_FP32_TRAIL, gp.GP_BF16_TRAIL])
def test_c4_mixed_against_oracle(c4, prec):
    g = c4
    r = gp.loglik(dev(g["X"]), dev(g["y"]), th_of(g), prec=prec, want_alpha=True)
    assert int(r["info"].item()) == 0
    ll, ld, q = r["out3"].cpu().numpy()
    ir = r["ir"].cpu().numpy()
    e = abs(ll - g["loglik"]) / abs(g["loglik"])
    a = r["alpha"].cpu().numpy()[g["a_idx"]]
    ea = np.linalg.norm(a - g["a_val"]) / np.linalg.norm(g["a_val"])
    print("prec %d n=32768: rel loglik err %.2e (logdet %.2e, q %.2e), alpha %.2e, ir %s" % (
        prec, e, abs(ld - g["logdet"]) / abs(g["logdet"]), abs(q - g["q"]) / abs(g["q"]), ea, ir))
    assert ir[2] == 1.0 and ir[1] <= 1e-10, ir
    assert e <= 1e-6
    assert math.isfinite(ll)
