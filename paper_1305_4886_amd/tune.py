"""Measure the library's tunable choices on this GPU and write the tuning table.

    python -m paper_1305_4886_amd.tune [--out PATH] [--sizes 4096,8192,...] [--quick] [--batched-only]

For each precision (FP64 and the FP32 / BF16 trailing-update modes) and each
size, gp_tune_potrf times the factorisation for every candidate panel width
and, in FP64, both K-slab shapes of the 128 x 128 trailing-update tile, and
records the fastest in the handle's table under the size bucket
floor(log2 n); gp_tune_batched times the schedules of the batched call (the
launch grid and the tile edge) for a batch of 64 problems with sizes uniform
on [256, 4096].  --batched-only keeps the factorisation entries of the
existing table and measures the batched call alone.  The table is then
written (default: the package's tuning.txt, which every handle loads when it
is created; entries of another architecture are ignored there).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    ap.add_argument("--sizes", default="2048,4096,8192,16384,32768,65536")
    ap.add_argument("--quick", action="store_true", help="fewer panel widths")
    ap.add_argument("--batched-only", action="store_true", help="re-measure the batched call only")
    a = ap.parse_args(argv)
    import torch

    import paper_1305_4886_amd as gp
    from paper_1305_4886_amd import synth

    h = gp.handle()
    if not a.batched_only:
        h.tune_clear()  # measure from scratch, not on top of a loaded table
    sizes = [] if a.batched_only else [int(v) for v in a.sizes.split(",") if v]
    # FP32 trailing updates stop at 768: each FP32 product sums K terms before it
    # meets the FP64 tile, and the 8-theta workload at n = 67,275 sits within a
    # factor of two of the 1e-6 loglik bar already; the split BF16 products are
    # two orders of magnitude inside it
    widths = {gp.GP_FP64: [384, 512, 640, 768, 896, 1024], gp.GP_FP32_TRAIL: [384, 512, 640, 768],
              gp.GP_BF16_TRAIL: [384, 512, 640, 768, 896, 1024]}
    if a.quick:
        widths = {p: w[1:3] for p, w in widths.items()}
    tail = 512  # the automatic tail width (gp_options_t.tail_nb = 0)
    for n in sizes:
        for prec, cand in widths.items():
            # a width above the tail width whose panels would all be the tail width
            # (n <= 24 x tail) runs the same schedule as the tail width itself
            cand = [w for w in cand if w <= tail or n > 24 * tail] or cand[:1]
            ms = h.tune_potrf(n, prec, nb=cand, panel_cus=(0,))
            o = h.options()
            print("n=%d prec=%d: %s -> nb %d slab %d" % (n, prec, {k[0]: round(v, 2) for k, v in ms.items()}, o.nb,
                                                        o.syrk_slab), flush=True)
            h.set_options(nb=0, syrk_slab=0, panel_cus=0)  # the table, not the options, carries the choice
            torch.cuda.empty_cache()
    # the batched call: 64 problems, sizes uniform on [256, 4096]
    sizes_b = synth.batch_sizes(64, 40)
    X = torch.as_tensor(np.concatenate([synth.uniform_points(int(k), 4000 + b) for b, k in enumerate(sizes_b)]),
                        device="cuda")
    y = torch.as_tensor(np.concatenate([synth.smooth_field(synth.uniform_points(int(k), 4000 + b), 5000 + b,
                                                           ell=0.1, t2=0.1) for b, k in enumerate(sizes_b)]),
                        device="cuda")
    th = gp.theta(gp.GP_EXP, 1.0, 0.1, 0.1)
    r = h.tune_batched(X, y, [th] * len(sizes_b), sizes_b)
    print("batched: %s -> grid %d tile %d" % (r, h.options().batch_grid, h.options().batch_tile), flush=True)
    h.set_options(batch_grid=0, batch_tile=0)
    h.tune_save(a.out)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
