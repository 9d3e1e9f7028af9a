"""Contrast histograms per quadtree step and pool size (Sec. 3.2 Fig 5,
Sec. 3.2.1 Fig 6) on synthetic images, with a contrast search over a
10-member set sampled from [0, 1] (the set the paper's earlier algorithms
searched): for the ranges accepted at each step, the chosen s and the
least-squares s* (Eq 2) of the chosen match.

    python -m paper_1502_00324_amd.s_histogram --size 512 --images 4 --pools 256,64,32
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--images", type=int, default=4)
    ap.add_argument("--pools", default="256,64,32", help="pool sizes DN")
    ap.add_argument("--split-rms", type=int, default=8)
    ap.add_argument("--nbins", type=int, default=10)
    ap.add_argument("--json", action="store_true", help="print one JSON object instead of tables")
    args = ap.parse_args()

    import torch

    from . import fic
    from .synth import make_image

    levels = [(16, 4), (8, 4), (4, 4), (2, 4)]
    s_num, s_den = list(range(1, 11)), 10
    ctx = fic.Context(0)
    imgs = [torch.from_numpy(make_image(100 + i, args.size, args.size, 40)).cuda() for i in range(args.images)]
    result = {}
    for dn in [int(v) for v in args.pools.split(",")]:
        p = fic.make_params(levels, pct=(0, 1), pool_max=dn, s_num=s_num, s_den=s_den,
                            split_rms=(args.split_rms, 1))
        acc = None
        for (pools, codes), t in zip(ctx.encode(imgs, p), imgs):
            h = ctx.s_histogram(t, p, pools, codes, args.nbins)
            if acc is None:
                acc = h
            else:
                for a, b in zip(acc, h):
                    for k in ("s_star", "s_index"):
                        a[k] = a[k] + b[k]
                    for k in ("under", "over", "flat"):
                        a[k] += b[k]
        result[dn] = [{k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in lv.items()} for lv in acc]
    ctx.close()
    if args.json:
        print(json.dumps({"size": args.size, "images": args.images, "s_set": [v / s_den for v in s_num],
                          "nbins": args.nbins, "histograms": result}))
        return
    for dn, per_step in result.items():
        print("pool size DN = %d" % dn)
        for l, h in enumerate(per_step):
            n = sum(h["s_index"])
            if n == 0:
                continue
            chosen = " ".join("%5.1f" % (100.0 * c / n) for c in h["s_index"])
            print("  step %d (%2dx%-2d, %6d ranges)  chosen s=%s %%: %s" %
                  (l + 1, levels[l][0], levels[l][0], n, ",".join("%.1f" % (v / s_den) for v in s_num), chosen))
            star = " ".join("%5.1f" % (100.0 * c / n) for c in [h["under"]] + h["s_star"] + [h["over"]])
            print("  %-38s s* <0 | %d bins of [0,1) | >=1 %%: %s  (flat %d)" % ("", args.nbins, star, h["flat"]))


if __name__ == "__main__":
    main()
