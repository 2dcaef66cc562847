"""Benchmark of the GP marginal-likelihood hot path on one MI355X.

Workload: n = 32768 points uniform on [0, 1]^2 (seed 4), exponential
covariance sigma^2 = 1, rho = 0.1, tau^2 = 0.1, synthetic response (smooth
random field + nugget noise).  One step = one pass over the hot path:
  * C(theta) build + blocked Cholesky (FP64)          -> Cholesky TFLOP/s
  * log-likelihood evaluation (FP64)                   -> evals/s
  * log-likelihood + adjoint gradient (FP64)           -> evals/s
  * mixed-precision log-likelihood (FP32 / BF16 trailing products + FP64
    refinement), with its error against the FP64 result -> evals/s; BF16
    with hi/lo split operands (default) and, for context, without
  * kriging mean + variance at m = 4096 new points     -> predictions/s
  * full m x m prediction covariance, and 1000 realizations conditional
    on the data at the m points                        -> TFLOP/s, draws/s
  * batch of 64 independent GPs, n_b uniform in [256, 4096], one launch
All inputs are resident in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N]

Prints one JSON line.  `value` is the FP64 Cholesky rate (n^3/3 over the
measured factorisation time); the other figures ride along under `parts`.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--parts", default="krige,sim,grad,mixed,batch")
    ap.add_argument("--nreal", type=int, default=1000, help="realizations drawn by the simulation part")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-n", type=int, default=12288, help="oracle sample size (leading block)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (scale for HBM counters)")
    return ap.parse_args()


TRAFFIC_N = 32768  # the workload size the committed counter summary was taken at
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_syrk_dma_trailing_n%d_hbm_traffic.md" % TRAFFIC_N)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1305_4886_amd", "csrc", f) for f in ("k_gemm.hip", "internal.h")]


def kernel_sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n=TRAFFIC_N):
    """HBM bytes per trailing-SYRK launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a plain copy of
    known size), or None when the kernel sources changed since it was taken
    or the workload size is not the one it was taken at."""
    import re

    if n != TRAFFIC_N:
        return None, "counters taken at n = %d only" % TRAFFIC_N

    try:
        with open(TRAFFIC_FILE) as fh:
            txt = fh.read()
    except OSError:
        return None, "no counter summary"
    b = re.search(r"^traffic_bytes_per_launch = (\d+)$", txt, re.M)
    h = re.search(r"^kernel_sources_sha256 = ([0-9a-f]{64})$", txt, re.M)
    if not b or not h:
        return None, "counter summary unreadable"
    if h.group(1) != kernel_sources_sha256():
        return None, "kernel sources changed since the counters were taken"
    return int(b.group(1)), "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, copy-calibrated"


def cpu_baseline(n_s, X_np, y_np, gpu_loglik=None):
    """The oracle's FP64 log-likelihood (covariance, Cholesky-Crout, both
    substitutions, compensated log-determinant and quadratic form) on the
    leading n_s points of the benchmark workload, timed on the host cores.
    Reported as its Cholesky rate (n_s^3 / 3 over the whole evaluation) and
    as evaluations per second at n_s and, scaled by n^3, at the full n; the
    GPU's log-likelihood of the same sample is compared with it."""
    import numpy as np

    import oracle

    oracle.build()
    n = X_np.shape[0]
    X = np.ascontiguousarray(X_np[:n_s])
    y = np.ascontiguousarray(y_np[:n_s])
    th = np.array([0.0, math.log(0.1), math.log(0.1)])
    t0 = time.perf_counter()
    ll, ld, q = oracle.loglik(0, th, X, y)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": n_s ** 3 / 3 / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": "oracle FP64 log-likelihood (covariance + Cholesky-Crout + substitutions + log-determinant) "
                     "of the leading %d points of the n=%d exponential workload: %.2f s" % (n_s, n, dt),
           "seconds": dt, "evals_per_s_sample": 1.0 / dt,
           "evals_per_s_at_n_extrapolated": 1.0 / (dt * (n / n_s) ** 3), "oracle_loglik_sample": ll}
    if gpu_loglik is not None:
        g = gpu_loglik(X, y)
        out["gpu_loglik_sample"] = g
        out["gpu_rel_err_sample"] = abs(g - ll) / abs(ll)
    return out


def golden_value(n):
    """The oracle's stored log-likelihood of the full workload (written by the
    golden-value script from the oracle alone), or None."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "exp_n%d.npz" % n)
    if not os.path.exists(path):
        return None
    d = np.load(path, allow_pickle=False)
    return {"loglik": float(d["loglik"]), "logdet": float(d["logdet"]), "q": float(d["q"]),
            "oracle_seconds": float(d["oracle_loglik_seconds"]) if "oracle_loglik_seconds" in d.files else None,
            "oracle_threads": int(d["oracle_threads"]) if "oracle_threads" in d.files else None}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (requested --gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1305_4886_amd as gp
    from paper_1305_4886_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 8, "launches": 3}))
        return
    dev = "cuda"
    n, m = a.n, a.m
    parts = set(a.parts.split(","))
    X_np = synth.uniform_points(n, 4)
    y_np = synth.smooth_field(X_np, 40, s2=1.0, ell=0.1, t2=0.1)
    X = torch.as_tensor(X_np, device=dev)
    y = torch.as_tensor(y_np, device=dev)
    th = gp.theta(gp.GP_EXP, 1.0, 0.1, 0.1)
    h = gp.handle()
    S = gp.colmajor_storage(n)
    ws_p = h.workspace(gp.GP_OP_POTRF, n)
    ws_l = h.workspace(gp.GP_OP_LOGLIK, n)
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = fn()
        e1.record(stream)
        return r, (e0, e1)

    results = {k: [] for k in ["chol", "loglik", "krige", "kcov", "sim", "grad", "mixed32", "mixed16", "mixed16s",
                               "batch"]}
    syrk = [0, 0.0, 0.0, 0.0]
    last = {}
    Xs = torch.as_tensor(synth.uniform_points(m, 41), device=dev)
    ws_k = h.workspace(gp.GP_OP_KRIGE, n, m) if "krige" in parts else None
    if "sim" in parts:
        # full prediction covariance and conditional realizations at the m new
        # points (1000 draws, as in the paper's example), seeded normals
        ws_kc = h.workspace(gp.GP_OP_KRIGE_COV, n, m)
        ws_sim = h.workspace(gp.GP_OP_SIMULATE, n, m)
        P_kc = gp.colmajor_storage(m)
        S_sim = gp.colmajor_storage(m)
        gen = torch.Generator(device=dev)
        gen.manual_seed(1000)
        eps = torch.randn((a.nreal, m), dtype=torch.float64, device=dev, generator=gen)
    ws_g = h.workspace(gp.GP_OP_LOGLIK_GRAD, n) if "grad" in parts else None
    ws_m32 = h.workspace(gp.GP_OP_LOGLIK, n, 0, gp.GP_FP32_TRAIL) if "mixed" in parts else None
    ws_m16 = h.workspace(gp.GP_OP_LOGLIK, n, 0, gp.GP_BF16_TRAIL) if "mixed" in parts else None
    if "batch" in parts:
        bsizes = synth.batch_sizes(64, 40)
        bX = torch.as_tensor(np.concatenate([synth.uniform_points(int(k), 4000 + b) for b, k in enumerate(bsizes)]),
                             device=dev)
        by = torch.as_tensor(np.concatenate([synth.smooth_field(synth.uniform_points(int(k), 4000 + b), 5000 + b,
                                                                ell=0.1, t2=0.1) for b, k in enumerate(bsizes)]),
                             device=dev)
        bth = [th] * len(bsizes)
        ws_b = h.workspace(gp.GP_OP_BATCHED, int(bsizes.max()), len(bsizes))
        bpool = torch.empty(int((bsizes.astype(np.int64) ** 2).sum()), dtype=torch.float64, device=dev)

    def step(record):
        # 1. covariance + FP64 Cholesky (timed: the factorisation only)
        gp.cov_build(X, th, S)
        if record:
            h.profile(True)
        info, ev = timed(lambda: gp.potrf(S, n, ws=ws_p))
        if record:
            results["chol"].append(ev)
            torch.cuda.synchronize()
            launches, ms, fl, alg = h.profile_read()
            h.profile(False)
            syrk[0] += launches
            syrk[1] += ms
            syrk[2] += fl
            syrk[3] += alg
            assert int(info.item()) == 0
        # 2. FP64 log-likelihood evaluation (cov build + Cholesky + solves + logdet), alpha kept
        r, ev = timed(lambda: gp.loglik(X, y, th, S=S, ws=ws_l, want_alpha=True))
        if record:
            results["loglik"].append(ev)
            last["loglik"] = r
        # 3. kriging mean + variance at m new points from that factor
        if "krige" in parts:
            kr, ev = timed(lambda: gp.krige(X, Xs, S, r["alpha"], th, ws=ws_k))
            if record:
                results["krige"].append(ev)
                last["krige"] = kr
        # 3b. full prediction covariance, conditional simulation
        if "sim" in parts:
            _, ev = timed(lambda: gp.krige_cov(X, Xs, S, th, out=P_kc, ws=ws_kc))
            if record:
                results["kcov"].append(ev)
            sm, ev = timed(lambda: gp.simulate(Xs, th, eps, X=X, S_data=S, alpha=r["alpha"], S=S_sim, ws=ws_sim))
            if record:
                results["sim"].append(ev)
                last["sim"] = sm
        # 4. log-likelihood + adjoint gradient (FP64)
        if "grad" in parts:
            g, ev = timed(lambda: gp.loglik_grad(X, y, th, S=S, ws=ws_g))
            if record:
                results["grad"].append(ev)
                last["grad"] = g
        # 5. mixed precision (FP32 / BF16 trailing products, FP64 refinement)
        if "mixed" in parts:
            m32, ev = timed(lambda: gp.loglik(X, y, th, prec=gp.GP_FP32_TRAIL, S=S, ws=ws_m32))
            if record:
                results["mixed32"].append(ev)
                last["mixed32"] = m32
            m16, ev = timed(lambda: gp.loglik(X, y, th, prec=gp.GP_BF16_TRAIL, S=S, ws=ws_m16))
            if record:
                results["mixed16"].append(ev)
                last["mixed16"] = m16
            # the same with one BF16 product per block (no hi / lo split), for context
            h.set_options(bf16_split=0)
            m16s, ev = timed(lambda: gp.loglik(X, y, th, prec=gp.GP_BF16_TRAIL, S=S, ws=ws_m16))
            h.set_options(bf16_split=1)
            if record:
                results["mixed16s"].append(ev)
                last["mixed16s"] = m16s
        # 6. batch of 64 independent GPs in one call
        if "batch" in parts:
            bb, ev = timed(lambda: gp.loglik_batched(bX, by, bth, bsizes, C_pool=bpool, ws=ws_b))
            if record:
                results["batch"].append(ev)
                last["batch"] = bb

    for _ in range(a.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def ms_of(evs):
        return [e0.elapsed_time(e1) for e0, e1 in evs]

    chol_ms = ms_of(results["chol"])
    t_chol = float(np.median(chol_ms)) / 1e3
    flops = n ** 3 / 3.0
    value = flops / t_chol / 1e12
    out_parts = {"cholesky_fp64": {"ms_median": t_chol * 1e3, "ms_min": min(chol_ms), "tflops": value,
                                   "frac_fp64_peak": value / FP64_PEAK_TFLOPS}}
    lm = ms_of(results["loglik"])
    ref = last["loglik"]["out3"].cpu().numpy().tolist()
    out_parts["loglik_fp64"] = {"ms_median": float(np.median(lm)), "evals_per_s": 1e3 / float(np.median(lm)),
                                "loglik": ref[0], "logdet": ref[1], "q": ref[2]}
    gold = golden_value(n)
    if gold is not None:
        out_parts["loglik_fp64"]["rel_err_vs_oracle"] = abs(ref[0] - gold["loglik"]) / abs(gold["loglik"])
        out_parts["oracle_full_n"] = {"loglik": gold["loglik"], "seconds": gold["oracle_seconds"],
                                      "threads": gold["oracle_threads"],
                                      "note": "oracle FP64 log-likelihood of the full workload, measured once by "
                                              "tests/golden/make_golden.py (not on this host)"}
    if results["krige"]:
        km = float(np.median(ms_of(results["krige"])))
        mean, var = last["krige"]
        out_parts["krige_fp64"] = {"m": m, "ms_median": km, "predictions_per_s": m / km * 1e3,
                                   "trsm_tflops": n * n * m / (km / 1e3) / 1e12,
                                   "var_min": float(var.min().item()), "var_max": float(var.max().item())}
    if results["kcov"]:
        cm = float(np.median(ms_of(results["kcov"])))
        sm = float(np.median(ms_of(results["sim"])))
        # flops: the right-side solve n^2 m, the SYRK m^2 n (lower half); the
        # simulation adds the factor m^3 / 3 and the product m^2 nreal
        kc_fl = n * n * m + m * m * n
        sim_fl = kc_fl + m ** 3 / 3 + m * m * a.nreal
        out_parts["krige_cov_fp64"] = {"m": m, "ms_median": cm, "tflops": kc_fl / (cm / 1e3) / 1e12}
        out_parts["simulate_cond_fp64"] = {"m": m, "realizations": a.nreal, "ms_median": sm,
                                           "tflops": sim_fl / (sm / 1e3) / 1e12,
                                           "realizations_per_s": a.nreal / sm * 1e3,
                                           "info": int(last["sim"]["info"].item())}
    if results["grad"]:
        gm = float(np.median(ms_of(results["grad"])))
        g = last["grad"]
        out_parts["loglik_grad_fp64"] = {"ms_median": gm, "evals_per_s": 1e3 / gm,
                                         "grad": g["grad"].cpu().numpy().tolist(),
                                         "loglik": float(g["out3"][0].item())}
    for key, name in [("mixed32", "loglik_mixed_fp32"), ("mixed16", "loglik_mixed_bf16"),
                      ("mixed16s", "loglik_mixed_bf16_unsplit")]:
        if results[key]:
            mm = float(np.median(ms_of(results[key])))
            r = last[key]
            llm = float(r["out3"][0].item())
            ir = r["ir"].cpu().numpy().tolist()
            out_parts[name] = {"ms_median": mm, "evals_per_s": 1e3 / mm, "loglik": llm,
                               "rel_err_vs_fp64": abs(llm - ref[0]) / abs(ref[0]),
                               "rel_err_vs_oracle": (abs(llm - gold["loglik"]) / abs(gold["loglik"])
                                                     if gold is not None else None),
                               "speedup_vs_fp64_eval": float(np.median(lm)) / mm,
                               "ir_sweeps": ir[0], "ir_rel_residual": ir[1], "ir_converged": bool(ir[2] == 1.0)}
            # the mixed form's bar: loglik within 1e-6 of the FP64 value, solve refined to 1e-10
            err = out_parts[name]["rel_err_vs_oracle"]
            err = out_parts[name]["rel_err_vs_fp64"] if err is None else err
            out_parts[name]["within_tolerance"] = bool(err <= 1e-6 and ir[1] <= 1e-10 and ir[2] == 1.0)
    if results["batch"]:
        bm = float(np.median(ms_of(results["batch"])))
        bflops = float((bsizes.astype(np.float64) ** 3).sum() / 3.0)
        out_parts["batch_fp64"] = {"problems": int(len(bsizes)), "ms_median": bm,
                                   "evals_per_s": len(bsizes) / bm * 1e3, "cholesky_tflops": bflops / (bm / 1e3) / 1e12,
                                   "all_finite": bool(torch.isfinite(last["batch"]["out3"]).all().item())}
    syrk_tflops = syrk[2] / (syrk[1] / 1e3) / 1e12 if syrk[1] > 0 else None
    syrk_per_launch_flops = syrk[2] / syrk[0] if syrk[0] else None
    traffic, traffic_src = measured_traffic(n)
    # algorithmic HBM bytes of the same launches (from the library's count): the
    # lower-triangle C entries read and written once, 8 B each way
    alg_bytes = syrk[3] / syrk[0] if syrk[0] else None
    roofline = {"kernel": "trailing SYRK (k_syrk_dma<2,16,1,x4,8 waves>, role 1)", "bound": "mfma",
                "achieved": syrk_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": (syrk_tflops / FP64_PEAK_TFLOPS) if syrk_tflops else None,
                "traffic": traffic, "traffic_unit": "B/launch", "traffic_source": traffic_src,
                "algorithmic_c_bytes_per_launch": alg_bytes, "launches": syrk[0],
                "avg_launch_ms": syrk[1] / syrk[0] if syrk[0] else None,
                "flops_per_launch": syrk_per_launch_flops}
    cpu = None
    if not a.no_cpu:
        def gpu_sample(Xc, yc):
            rr = gp.loglik(torch.as_tensor(Xc, device=dev), torch.as_tensor(yc, device=dev), th)
            return float(rr["out3"][0].item())

        cpu = cpu_baseline(a.cpu_n, X_np, y_np, gpu_sample)
    line = {
        "metric": "Cholesky TFLOP/s + loglik(+grad) evals/s at n=32768: mixed vs FP64",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "exp_n%d" % n, "n": n, "points": "uniform [0,1]^2 seed 4", "batch": "64 GPs, n_b uniform on [256, 4096] (seed 40)",
                   "kernel": "exponential", "sigma2": 1.0, "rho": 0.1, "tau2": 0.1, "m": m,
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "parts": out_parts,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
