"""Batched likelihoods: each problem of a ragged batch must match the
single-problem CPU oracle (same model and definitions, Section 1), including
per-problem failure reporting.  Every schedule is covered: the persistent
launch on 128- and on 64-wide tiles, each with its automatic grid, with one
workgroup (every task in ticket order on one workgroup) and with a small odd
grid, and the level-synchronous launches."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1305_4886_amd as gp  # noqa: E402
from paper_1305_4886_amd import synth  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


def make_batch(sizes, seed, kernels=None):
    Xs, ys, ths = [], [], []
    for b, n in enumerate(sizes):
        X = synth.uniform_points(int(n), seed + b)
        y = synth.smooth_field(X, seed + 1000 + b, ell=0.1, t2=0.1) if n > 0 else np.zeros(0)
        k = kernels[b] if kernels else b % 3
        th = np.array([math.log(1.0 + 0.1 * (b % 3)), math.log(0.1), math.log(0.1)])
        Xs.append(X); ys.append(y); ths.append((k, th))
    return Xs, ys, ths


# (batch_grid, batch_tile): persistent launches (one workgroup per compute
# unit, one workgroup, seven workgroups) with 128- and 64-wide tiles, and the
# level-synchronous launches
GRIDS = [(0, 128), (1, 128), (7, 128), (0, 64), (1, 64), (7, 64), (-1, 0)]


@pytest.fixture(params=GRIDS, ids=lambda g: "grid%d_tile%d" % g)
def grid(request):
    h = gp.handle()
    saved = h.options()
    h.set_options(batch_grid=request.param[0], batch_tile=request.param[1])
    yield request.param
    h.set_options(batch_grid=saved.batch_grid, batch_tile=saved.batch_tile)


@pytest.mark.parametrize("sizes", [[1], [64], [65, 3, 200], [300, 0, 129, 1000, 64, 777, 511, 2]])
def test_batched_matches_oracle(orc, sizes, grid):
    Xs, ys, ths = make_batch(sizes, 70)
    X = np.concatenate([x for x in Xs if len(x)] or [np.zeros((0, 2))])
    y = np.concatenate([v for v in ys if len(v)] or [np.zeros(0)])
    r = gp.loglik_batched(dev(X), dev(y), [gp.theta(k, log=t) for k, t in ths], sizes)
    out = r["out3"].cpu().numpy()
    info = r["info"].cpu().numpy()
    for b, n in enumerate(sizes):
        assert info[b] == 0
        if n == 0:
            assert np.all(out[b] == 0.0)
            continue
        k, t = ths[b]
        ll, ld, q = orc.loglik(k, t, Xs[b], ys[b])
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (b, n, out[b], ll)
        assert abs(out[b, 1] - ld) <= 1e-11 * max(1.0, abs(ld))


def test_batched_factor_in_pool(orc, grid):
    """On return each problem's slice of the pool holds its lower factor."""
    sizes = [200, 64, 131]
    Xs, ys, ths = make_batch(sizes, 80)
    r = gp.loglik_batched(dev(np.concatenate(Xs)), dev(np.concatenate(ys)),
                          [gp.theta(k, log=t) for k, t in ths], sizes)
    pool = r["C_pool"].cpu().numpy()
    off = 0
    for b, n in enumerate(sizes):
        k, t = ths[b]
        Lg = np.tril(pool[off:off + n * n].reshape(n, n).T)
        Lo, oinfo = orc.potrf(orc.cov(k, t, Xs[b]))
        assert oinfo == 0
        assert np.linalg.norm(Lg - Lo) <= 1e-12 * np.linalg.norm(Lo), b
        off += n * n


def test_batched_more_than_64_tile_columns(orc, grid):
    """n = 4200 has 66 tile columns: the dependency polls span more than one wave's width."""
    sizes = [4200, 100]
    Xs, ys, ths = make_batch(sizes, 85, kernels=[1, 0])
    r = gp.loglik_batched(dev(np.concatenate(Xs)), dev(np.concatenate(ys)),
                          [gp.theta(k, log=t) for k, t in ths], sizes)
    out = r["out3"].cpu().numpy()
    assert np.all(r["info"].cpu().numpy() == 0)
    for b in range(2):
        k, t = ths[b]
        ll, ld, q = orc.loglik(k, t, Xs[b], ys[b])
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (b, out[b], ll)
        assert abs(out[b, 2] - q) <= 1e-11 * abs(q)


_BIG = {}


def test_batched_more_than_64_wide_tile_columns(orc, grid):
    """n = 8300 has 65 tile columns of 128: the dependency polls of the
    128-wide tiles also span more than one wave's width."""
    if grid[0] < 0 or grid[1] != 128:
        pytest.skip("128-wide tiles only")
    sizes = [8300, 130]
    Xs, ys, ths = make_batch(sizes, 87, kernels=[0, 2])
    if not _BIG:
        _BIG.update({b: orc.loglik(ths[b][0], ths[b][1], Xs[b], ys[b]) for b in range(2)})
    r = gp.loglik_batched(dev(np.concatenate(Xs)), dev(np.concatenate(ys)),
                          [gp.theta(k, log=t) for k, t in ths], sizes)
    out = r["out3"].cpu().numpy()
    assert np.all(r["info"].cpu().numpy() == 0)
    for b in range(2):
        ll, ld, q = _BIG[b]
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (b, out[b], ll)
        assert abs(out[b, 1] - ld) <= 1e-11 * abs(ld)
        assert abs(out[b, 2] - q) <= 1e-11 * abs(q)


def test_batched_workload_64_problems(orc):
    sizes = synth.batch_sizes(64, 40)
    Xs, ys, ths = make_batch(sizes, 4000, kernels=[0] * 64)
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    r = gp.loglik_batched(dev(X), dev(y), [gp.theta(k, log=t) for k, t in ths], sizes)
    out = r["out3"].cpu().numpy()
    assert np.all(r["info"].cpu().numpy() == 0)
    # every problem against the oracle (about 4e11 flops of oracle Cholesky)
    worst = 0.0
    for b in range(len(sizes)):
        k, t = ths[b]
        ll, ld, q = orc.loglik(k, t, Xs[b], ys[b])
        worst = max(worst, abs(out[b, 0] - ll) / abs(ll))
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (b, sizes[b], out[b], ll)
        assert abs(out[b, 1] - ld) <= 1e-11 * abs(ld), b
        assert abs(out[b, 2] - q) <= 1e-11 * abs(q), b
    print("64 problems: worst relative loglik difference %.2e" % worst)


def test_batched_failure_is_per_problem(grid):
    sizes = [100, 150, 80]
    Xs, ys, ths = make_batch(sizes, 90, kernels=[0, 0, 0])
    Xs[1][120] = Xs[1][30]  # duplicate point, no nugget -> not PD
    ths[1] = (0, np.array([0.0, math.log(0.3), -np.inf]))
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    r = gp.loglik_batched(dev(X), dev(y), [gp.theta(k, log=t) for k, t in ths], sizes)
    out = r["out3"].cpu().numpy()
    info = r["info"].cpu().numpy()
    assert info[0] == 0 and info[2] == 0
    assert np.all(np.isfinite(out[0])) and np.all(np.isfinite(out[2]))
    if info[1] != 0:
        assert info[1] >= 121 and np.all(np.isnan(out[1]))


def test_tune_batched_picks_a_candidate(orc):
    """The schedule autotuner times every candidate, keeps the fastest, and the
    kept schedule still matches the oracle."""
    sizes = [300, 129, 64, 700]
    Xs, ys, ths = make_batch(sizes, 95, kernels=[0, 1, 2, 0])
    X, y = dev(np.concatenate(Xs)), dev(np.concatenate(ys))
    thetas = [gp.theta(k, log=t) for k, t in ths]
    h = gp.handle()
    saved = h.options()
    try:
        ms = h.tune_batched(X, y, thetas, sizes, grids=(-1, 0, 5, 0), tiles=(0, 64, 128, 128))
        assert set(ms) == {(-1, 0), (0, 64), (5, 128), (0, 128)} and all(v > 0 for v in ms.values()), ms
        best = min(ms, key=ms.get)
        assert h.options().batch_grid == best[0]
        assert best[0] < 0 or h.options().batch_tile == best[1]
        out = gp.loglik_batched(X, y, thetas, sizes)["out3"].cpu().numpy()
        for b in range(len(sizes)):
            k, t = ths[b]
            ll, _, _ = orc.loglik(k, t, Xs[b], ys[b])
            assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll)
    finally:
        h.set_options(batch_grid=saved.batch_grid, batch_tile=saved.batch_tile)
        h.tune_reset()


def test_batched_many_theta_over_shared_points(orc, grid):
    """Many theta over one point set: every problem names the same points
    (equal point offsets) with its own parameters and kernel."""
    n = 333
    X = synth.uniform_points(n, 97)
    y = synth.smooth_field(X, 98, ell=0.1, t2=0.1)
    ths = []
    for b in range(6):
        th = np.array([math.log(0.5 + 0.3 * b), math.log(0.05 + 0.03 * b), math.log(0.02 + 0.05 * b)])
        ths.append((b % 3, th))
    sizes = [n] * len(ths)
    r = gp.loglik_batched(dev(X), dev(y), [gp.theta(k, log=t) for k, t in ths], sizes,
                          x_off=[0] * len(ths))
    out = r["out3"].cpu().numpy()
    assert np.all(r["info"].cpu().numpy() == 0)
    for b, (k, t) in enumerate(ths):
        ll, ld, q = orc.loglik(k, t, X, y)
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (b, out[b], ll)
        assert abs(out[b, 2] - q) <= 1e-11 * abs(q)


@pytest.mark.parametrize("dim", [1, 3])
def test_batched_other_point_dimensions(orc, grid, dim):
    """Points on a line (dim 1) and in space (dim 3): the persistent launches
    take their coordinates through the general distance path, not the planar
    one staged in LDS."""
    sizes = [130, 257, 64, 1]
    rng = np.random.default_rng(70 + dim)
    Xs = [rng.uniform(0.0, 1.0, size=(n, dim)) for n in sizes]
    ys = [rng.standard_normal(n) for n in sizes]
    ths = [(b % 3, np.array([math.log(1.0 + 0.2 * b), math.log(0.2), math.log(0.05)])) for b in range(len(sizes))]
    r = gp.loglik_batched(dev(np.concatenate(Xs)), dev(np.concatenate(ys)), [gp.theta(k, log=t) for k, t in ths],
                          sizes)
    out = r["out3"].cpu().numpy()
    assert np.all(r["info"].cpu().numpy() == 0)
    for b in range(len(sizes)):
        k, t = ths[b]
        ll, ld, q = orc.loglik(k, t, Xs[b], ys[b])
        assert abs(out[b, 0] - ll) <= 1e-11 * abs(ll), (dim, b, out[b], ll)
        assert abs(out[b, 1] - ld) <= 1e-11 * max(1.0, abs(ld)), (dim, b)
        assert abs(out[b, 2] - q) <= 1e-11 * abs(q), (dim, b)
