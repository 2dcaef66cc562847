"""The tuning table: the autotuner's choices are recorded per (operation,
precision, size bucket), written and read back as text, consulted by the
factorisation when the panel width is automatic, and tied to the device's
architecture.  Results stay those of the oracle whatever the table holds."""
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


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[case]", request.node.name, flush=True)
    yield
    torch.cuda.synchronize()


def ws_bytes(h, n, prec=gp.GP_FP64):
    b = ctypes.c_size_t()
    gp.check(gp.lib().gp_workspace_size(h.ptr, gp.GP_OP_POTRF, n, 0, prec, ctypes.byref(b)))
    return b.value


def arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def test_table_round_trip_and_lookup(tmp_path):
    h = gp.handle()
    saved = h.options()
    try:
        h.tune_clear()
        n = 1500  # size bucket 10: 1024 .. 2047
        default = ws_bytes(h, n)
        times = h.tune_potrf(n, nb=(128, 256), panel_cus=(0,))
        best_nb = min(times, key=times.get)[0]
        o = h.options()
        assert o.nb == best_nb and o.syrk_slab in (8, 16)
        h.set_options(nb=0, syrk_slab=0)
        path = str(tmp_path / "table.txt")
        h.tune_save(path)
        lines = [ln for ln in open(path) if not ln.startswith("#")]
        assert len(lines) == 1 and lines[0].split()[0] == arch()
        assert lines[0].split()[1:5] == ["0", "0", "10", str(best_nb)]
        h.tune_clear()
        assert ws_bytes(h, n) == default
        # entries of another architecture are skipped; this device's are merged
        with open(path, "a") as f:
            f.write("gfx000 0 0 10 64 0 8 0\n")
        assert h.tune_load(path) == 1
        h.set_options(nb=best_nb)
        tuned, tuned_1100 = ws_bytes(h, n), ws_bytes(h, 1100)
        h.set_options(nb=768)
        default_3000 = ws_bytes(h, 3000)
        h.set_options(nb=0)
        # the bucket 1024 .. 2047 takes the tuned width, bucket 2048 .. 4095 the default
        assert ws_bytes(h, n) == tuned and ws_bytes(h, 1100) == tuned_1100
        assert ws_bytes(h, 3000) == default_3000
        # the plan query reports the same resolution: tuned width in the bucket, default outside
        assert h.potrf_plan(n)[0] == best_nb and h.potrf_plan(1100)[0] == best_nb
        assert h.potrf_plan(3000) == (768, 0, 16, 512)
        # the factor with the tuned choice still matches the oracle
        X = synth.uniform_points(n, 5)
        t = np.array([0.0, math.log(0.1), math.log(0.1)])
        C = oracle.cov(0, t, X)
        S = gp.colmajor_storage(n)
        gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(C)))
        assert int(gp.potrf(S, n).item()) == 0
        Lo, _ = oracle.potrf(C)
        L = np.tril(S[:n, :n].T.cpu().numpy())
        assert np.linalg.norm(L - Lo) <= 1e-12 * np.linalg.norm(Lo)
    finally:
        h.set_options(nb=saved.nb, syrk_slab=saved.syrk_slab, panel_cus=saved.panel_cus)
        h.tune_reset()


def test_malformed_or_missing_table(tmp_path):
    h = gp.handle()
    bad = tmp_path / "bad.txt"
    bad.write_text("%s 0 0 10 100 0 8 0\n" % arch())  # a width that is not a multiple of 64
    with pytest.raises(gp.GPError) as e:
        h.tune_load(str(bad))
    assert e.value.code == -1008
    with pytest.raises(gp.GPError) as e:
        h.tune_load(str(tmp_path / "missing.txt"))
    assert e.value.code == -1008
    with pytest.raises(gp.GPError) as e:
        h.set_options(syrk_slab=12)
    assert e.value.code == -2
    for bad_tail in (-2, 100):
        with pytest.raises(gp.GPError) as e:
            h.set_options(tail_nb=bad_tail)
        assert e.value.code == -2


def test_shipped_table_is_for_this_device():
    import os
    if not os.path.exists(gp.TUNING_TABLE):
        pytest.skip("no shipped table")
    rows = [ln.split() for ln in open(gp.TUNING_TABLE) if ln.strip() and not ln.startswith("#")]
    assert rows and all(r[0] == "gfx950" for r in rows)
    h = gp.handle()
    assert h.tune_load(gp.TUNING_TABLE) == len(rows)
    h.tune_reset()


@pytest.mark.parametrize("slab", [8, 16])
def test_both_tile_shapes_factor_correctly(slab):
    # the two K-slab shapes of the trailing-update tile at the benchmark's
    # panel width, with ld = n (the 16-byte copies), against the oracle
    n = 3000
    X = synth.uniform_points(n, 8)
    t = np.array([0.0, math.log(0.05), math.log(0.01)])
    C = oracle.cov(1, t, X)
    h = gp.handle()
    saved = h.options()
    try:
        h.set_options(nb=768, syrk_slab=slab, tail_nb=-1)
        assert h.potrf_plan(n) == (768, 0, slab, 768)
        S = gp.colmajor_storage(n)
        gp.colmajor(S, n).copy_(torch.as_tensor(np.tril(C)))
        assert int(gp.potrf(S, n).item()) == 0
    finally:
        h.set_options(nb=saved.nb, syrk_slab=saved.syrk_slab, tail_nb=saved.tail_nb)
    Lo, _ = oracle.potrf(C)
    L = np.tril(S[:n, :n].T.cpu().numpy())
    err = np.linalg.norm(L - Lo) / np.linalg.norm(Lo)
    print("slab %d: factor rel err %.2e" % (slab, err))
    assert err <= 1e-12


def trailing_launches(n, nb, tail):
    """The trailing updates of a lookahead factorisation, as (M, N, K): the
    panel [c0, c1) updates the next panel's columns, then the rest."""
    def width(c):
        w = tail if (0 < tail < nb and n - c <= 24 * tail) else nb
        return min(w, n - c)
    out, c0, c1 = [], 0, width(0)
    while c1 < n:
        c2 = c1 + width(c1)
        out.append((n - c1, c2 - c1, c1 - c0))
        if c2 < n:
            out.append((n - c2, n - c2, c1 - c0))
        c0, c1 = c1, c2
    return out


@pytest.mark.parametrize("n,nb,tail", [(4000, 512, 128), (4096, 768, -1), (2000, 384, 0), (3001, 512, 0)])
def test_profile_counts_the_trailing_updates(n, nb, tail):
    # the profile read that the benchmark's roofline is computed from: one
    # launch per trailing update, 2 K E flops and 16 E bytes for E updated
    # lower-trapezoid entries, E = N M - N (N - 1) / 2
    X = synth.uniform_points(n, 9)
    t = np.array([0.0, math.log(0.1), math.log(0.1)])
    h = gp.handle()
    saved = h.options()
    S = gp.colmajor_storage(n)
    try:
        h.set_options(nb=nb, tail_nb=tail, lookahead=1)
        gp.cov_build(torch.as_tensor(X, device="cuda"), gp.theta(0, log=t), S)
        h.profile_read()  # drop anything counted before
        h.profile(True)
        info = gp.potrf(S, n)
        torch.cuda.synchronize()
        launches, ms, flops, nbytes = h.profile_read()
    finally:
        h.profile(False)
        h.set_options(nb=saved.nb, tail_nb=saved.tail_nb, lookahead=saved.lookahead)
    assert int(info.item()) == 0
    sched = trailing_launches(n, nb, tail if tail != 0 else 512)
    ent = [N * M - N * (N - 1) / 2 for M, N, K in sched]
    assert launches == len(sched)
    assert math.isclose(flops, sum(2 * K * e for (M, N, K), e in zip(sched, ent)), rel_tol=1e-12)
    assert math.isclose(nbytes, sum(16 * e for e in ent), rel_tol=1e-12)
    assert ms > 0.0
