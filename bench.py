#!/usr/bin/env python3
"""Throughput of the fractal encoder's range-to-domain search on one MI355X.

One step = one whole encode of the workload's images (every quadtree level:
pool build, operand preparation, search, per-range codes, child lists) with
the default matrix engines, inputs resident in HBM.  The default engine takes
the matrix form measured fastest per block size: f16 MFMA with 32x32 result
tiles at B = 2 and 4, f16 MFMA with 16x16 tiles at B = 8, int8 MFMA on the
decimated hi/lo planes at B = 16 and 32.  Every form is exact; the "dtype"
field lists the forms the run used and "config.engine" maps them to block
sizes.  The metric is range x domain x isometry comparisons per second: sum
over levels of searched ranges x pool domains x 8 per step, divided by the
step time.

Printed as one JSON line, with: the plain FP32 engine timed on the same
workload (its codes and pools compared with the matrix run field by field);
the roofline of the dominant kernel (the search of the level that takes
longest, its launches timed with HIP events recorded on the encode stream);
the CPU oracle timed on a bounded sample of the same workload; and a second
leg on the 4096 x 4096 workload (encode time, its dominant search against
the int8 peak, 8 decode iterations and PSNR) under the key "c5_4096".
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published dense peaks per engine dtype (TFLOP/s, int8 in TOPS)
PEAK = {"mfma_f16": 2500.0, "mfma_f16_16x16": 2500.0, "mfma_i8": 5000.0, "fp32": 157.3}
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1502_00324_amd/csrc/k_search_mfma.hip", "paper_1502_00324_amd/csrc/k_search_f16.hip",
                  "paper_1502_00324_amd/csrc/search_common.h", "paper_1502_00324_amd/csrc/fic_internal.h"]
CODE_FIELDS = ("xy", "split", "domain", "iso", "s_idx", "offset", "err")
POOL_FIELDS = ("xy", "key", "sum4", "a")


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", "traffic_search_%s.json" % workload)


def issued_ops(engine_name, B):
    """MFMA ops the engine issues per comparison (the algorithmic count is 2 B^2)."""
    if engine_name in ("mfma_f16", "mfma_f16_16x16"):
        return 2 * max(16, B * B)              # K = B^2 decimated positions (B = 2 padded to 16)
    if engine_name == "mfma_i8":
        return 8 * B * B if B == 4 else 4 * B * B   # raw pixels at B=4, hi/lo planes above
    return 2 * B * B


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def host_cpu():
    """CPU model and thread counts of the host running the oracle."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "usable_cpus": usable}


def level_counts(bufs, p, images):
    """(B, ranges, pool, searched ranges) per level and image, read back after
    a run.  Searched: every range but the constant ones when the level's S
    holds 0 (their code is fixed without a search)."""
    import numpy as np
    out = []
    for (pools, codes), img in zip(bufs, images):
        per = []
        f = img.astype(np.int64)
        for l in range(p.levels):
            B = p.block0 >> l
            R = int(codes[l].count.item())
            xy = codes[l].xy[:R].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            flat = 0
            if p.s_num[l][0] == 0 and R:
                x, y = xy & 0xFFFF, xy >> 16
                v = np.lib.stride_tricks.sliding_window_view(f, (B, B))[y, x].reshape(R, -1)
                flat = int((v.max(1) == v.min(1)).sum())
            per.append((B, R, int(pools[l].count.item()), R - flat))
        out.append(per)
    return out


def run_steps(ctx, imgs, p, bufs, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.encode(imgs, p, bufs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1)


def same_outputs(a_bufs, b_bufs, levels):
    """Every pool and code field of every level and image equal (device compare)."""
    for (pa, ca), (pb, cb) in zip(a_bufs, b_bufs):
        for l in range(levels):
            n = int(ca[l].count.item())
            if n != int(cb[l].count.item()):
                return False
            for f in CODE_FIELDS:
                if not bool((getattr(ca[l], f)[:n] == getattr(cb[l], f)[:n]).all()):
                    return False
            m = int(pa[l].count.item())
            if m != int(pb[l].count.item()):
                return False
            for f in POOL_FIELDS:
                if not bool((getattr(pa[l], f)[:m] == getattr(pb[l], f)[:m]).all()):
                    return False
    return True


def cpu_baseline(wl, images, counts, budget_s):
    """The oracle, single-threaded, on a bounded sample: full pool builds and
    a seeded sample of ranges per level, scaled to the whole workload."""
    import numpy as np

    import oracle
    oracle.build()
    seed, W, H, nrect = wl.images[0]
    img = images[0]
    rng = np.random.default_rng(7)
    total_triples, t_total, sampled = 0, 0.0, []
    per_level_budget = budget_s / max(1, len(wl.levels))
    for l, (B, L) in enumerate(wl.levels):
        t0 = time.perf_counter()
        pool = oracle.build_pool(img, B, L, wl.pct, wl.pool_max)
        t_pool = time.perf_counter() - t0
        s_num = list(wl.s_num[l]) if isinstance(wl.s_num[0], (tuple, list)) else list(wl.s_num)
        all_r = oracle.level0_ranges(W, H, B)
        done, t_search = 0, 0.0
        while t_search < per_level_budget - t_pool and done < len(all_r):
            pick = all_r[rng.integers(0, len(all_r), 2)]
            t1 = time.perf_counter()
            oracle.encode_level(img, pool["xy"], pick, B, s_num, wl.s_den if isinstance(wl.s_den, int)
                                else wl.s_den[l], wl.split_rms, l == len(wl.levels) - 1, workers=1)
            t_search += time.perf_counter() - t1
            done += len(pick)
        _, R, P, _ = counts[0][l]
        per_range = t_search / done
        t_total += t_pool + per_range * R
        total_triples += R * P * 8
        sampled.append("level %d (B=%d): full pool (%.2f s) + %d ranges x %d domains (%.2f s)" %
                       (l, B, t_pool, done, len(pool["xy"]), t_search))
    return {"value": total_triples / t_total, "unit": "comparisons/s", "cores": 1, "kind": "oracle",
            "sample": "; ".join(sampled) + "; time scaled to every range of the GPU run's levels",
            "extrapolated_encode_s": round(t_total, 2), **host_cpu()}


class Leg:
    """One workload encoded with one engine: buffers, tiles, timed steps."""

    def __init__(self, ctx, wl, engine, pool_key, dev, fic, torch):
        from paper_1502_00324_amd.synth import make_image
        self.ctx, self.wl, self.engine, self.fic, self.torch = ctx, wl, engine, fic, torch
        self.images = [make_image(s, w, h, n) for (s, w, h, n) in wl.images]
        self.imgs = [torch.from_numpy(im).to(dev) for im in self.images]
        self.mk = lambda e: fic.make_params(wl.levels, pct=wl.pct, pool_max=wl.pool_max, s_num=wl.s_num,
                                            s_den=wl.s_den, split_rms=wl.split_rms, engine=e, pool_key=pool_key)
        self.p = self.mk(engine)
        self.dev = dev
        self.bufs = ctx.alloc_encode(self.shapes(), self.p, dev)
        self.tiles = {}

    def shapes(self):
        return [(im.shape[1], im.shape[0]) for im in self.images]

    def engine_name(self, B, engine=None):
        fic = self.fic
        names = {fic.ENGINE_MFMA_F16: "mfma_f16", fic.ENGINE_MFMA_I8: "mfma_i8", fic.ENGINE_FP32: "fp32",
                 fic.ENGINE_MFMA_F16_16X16: "mfma_f16_16x16"}
        return names[fic.level_engine(self.engine if engine is None else engine, B)]

    def tune(self, autotune):
        fic = self.fic
        if autotune:
            self.ctx.autotune(self.imgs, self.p, self.bufs, reps=3)
        t = self.ctx.get_tuning()
        for (B, L) in self.wl.levels:
            name = self.engine_name(B)
            if name in fic.FORM_NAMES:
                f = fic.FORM_NAMES.index(name)
                c = max(0, t.choice[f][B.bit_length() - 1])
                self.tiles["B=%d" % B] = {"form": name, "candidate": c, "of": fic.shape_count(f, B),
                                          "pl_rq_dt_wpe": list(fic.shape_describe(f, B, c))}

    def time(self, steps, warmup, graphs=False):
        ctx, torch = self.ctx, self.torch
        if graphs:
            ctx.set_graphs(4)
        for _ in range(warmup):
            ctx.encode(self.imgs, self.p, self.bufs)
        torch.cuda.synchronize()
        if steps is None:
            # about five seconds of timed encodes (at least ten), so the GPU
            # phase is long enough to sample and its averages are steady
            one = run_steps(ctx, self.imgs, self.p, self.bufs, 2, torch)
            steps = max(10, min(2000, int(5.0 / max(one, 1e-6))))
        if graphs:
            # graph replays are timed as a whole; stage times need eager encodes
            sec = run_steps(ctx, self.imgs, self.p, self.bufs, steps, torch)
            ctx.set_graphs(0)
            ctx.set_timing(True)
            run_steps(ctx, self.imgs, self.p, self.bufs, steps, torch)
        else:
            ctx.set_timing(True)
            sec = run_steps(ctx, self.imgs, self.p, self.bufs, steps, torch)
        stages = ctx.read_timing()
        ctx.set_timing(False)
        self.sec, self.stages, self.steps = sec, stages, steps
        self.counts = level_counts(self.bufs, self.p, self.images)
        # comparisons the search kernels evaluate (ranges searched x pool x 8);
        # the exhaustive count also holds the constant ranges coded in closed form
        self.triples_by_B, self.exhaustive = {}, 0
        for per_img in self.counts:
            for (B, R, P, Rs) in per_img:
                self.triples_by_B[B] = self.triples_by_B.get(B, 0) + Rs * P * 8
                self.exhaustive += R * P * 8
        self.triples = sum(self.triples_by_B.values())
        return sec

    def roofline(self):
        """The search launch with the largest summed event time, against its dtype's dense peak."""
        search = {B: v for (name, B), v in self.stages.items() if name == "search"}
        dom_B = max(search, key=lambda b: search[b][0])
        ms_tot, launches = search[dom_B]
        avg_ms = ms_tot / launches
        launches_per_step = launches / max(self.steps, 1)
        dom_engine = self.engine_name(dom_B)
        alg_ops = self.triples_by_B[dom_B] * 2 * dom_B * dom_B / launches_per_step   # decimated MACs x 2
        achieved = alg_ops / (avg_ms * 1e-3) / 1e12
        peak = PEAK[dom_engine]
        traffic = self.committed_traffic(dom_B)
        issued = issued_ops(dom_engine, dom_B) / (2 * dom_B * dom_B)
        out = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
               "frac": round(achieved / peak, 4), "traffic": traffic,
               "kernel": "search B=%d (%s engine)" % (dom_B, dom_engine), "avg_launch_ms": round(avg_ms, 4),
               "ops_per_launch": alg_ops,
               "ops_note": "algorithmic ops = 2 B^2 per comparison (the decimated inner product); this engine "
                           "issues %gx that on the matrix cores (%.1f TFLOP/s issued), peak is the %s dense peak"
                           % (issued, issued * achieved, dom_engine.replace("mfma_", ""))}
        if traffic:
            out["hbm_frac"] = round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        return out

    def committed_traffic(self, dom_B):
        """HBM bytes per launch from the committed counter passes, when they
        were taken on these sources and on the kernel instantiation this run used."""
        tile = self.tiles.get("B=%d" % dom_B, {})
        sh = tile.get("pl_rq_dt_wpe")
        want = None
        if sh and tile.get("form") == "mfma_f16":
            want = "k_f16_search<%d, %d, %d, %d>" % ((dom_B * dom_B + 15) // 16, sh[1], sh[2], sh[3])
        elif sh:
            pl = sh[0]
            ka = {1: dom_B * dom_B // 16, 2: dom_B * dom_B // 64, 3: dom_B * dom_B // 32, 4: 1}[pl]
            want = "k_mfma_search<%d, %d, %d, %d, %d>" % (ka, pl, sh[1], sh[2], sh[3])
        tf = traffic_file(self.wl.name)
        if not (os.path.exists(tf) and want):
            return None
        with open(tf) as f:
            tr = json.load(f)
        det = tr.get("per_launch_detail", {}).get(str(dom_B), {})
        if tr.get("source_hash") == kernel_source_hash() and want in det.get("kernel", ""):
            return tr.get("per_launch_bytes", {}).get(str(dom_B))
        return None

    def stage_ms(self):
        return {"%s_B%d" % (n, B): round(v[0] / max(self.steps, 1), 4) for (n, B), v in sorted(self.stages.items())}

    def decode(self, iters, reps=3):
        """Decode each image (untimed by the step clock): mean ms over reps and PSNR (Eq 4)."""
        import numpy as np
        torch, ctx = self.torch, self.ctx
        outs = [ctx.decode(self.p, pools, codes, im.shape[1], im.shape[0], iters)
                for (pools, codes), im in zip(self.bufs, self.images)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            outs = [ctx.decode(self.p, pools, codes, im.shape[1], im.shape[0], iters)
                    for (pools, codes), im in zip(self.bufs, self.images)]
        torch.cuda.synchronize()
        dec_ms = (time.perf_counter() - t0) * 1e3 / reps
        px = sum(im.size for im in self.images)
        sse = sum(int(((o.cpu().numpy().astype(np.int64) - im.astype(np.int64)) ** 2).sum())
                  for o, im in zip(outs, self.images))
        return {"iterations": iters, "ms": round(dec_ms, 3),
                "psnr_db": round(10 * np.log10(65025.0 * px / sse), 3) if sse else float("inf")}

    def levels_json(self):
        if len(self.counts) != 1:
            return None
        return [{"B": B, "ranges": R, "ranges_searched": Rs, "pool": P, "comparisons": Rs * P * 8}
                for (B, R, P, Rs) in self.counts[0]]

    def dtype(self):
        return "+".join(sorted({self.engine_name(B).replace("mfma_", "") for (B, L) in self.wl.levels}))

    def engine_desc(self):
        return ", ".join("B=%d %s" % (B, self.engine_name(B)) for (B, L) in self.wl.levels)


def second_leg(fic, torch, dev, args):
    """The 4096 x 4096 workload: one smaller leg with the library's default
    tile shapes (measured fastest there), so the largest configuration has a
    timed number in the same JSON line."""
    from paper_1502_00324_amd.configs import WORKLOADS
    wl = WORKLOADS["c5_4096"]
    ctx = fic.Context(0)
    try:
        leg = Leg(ctx, wl, fic.ENGINE_MFMA, fic.POOL_ENTROPY, dev, fic, torch)
        leg.tune(False)
        sec = leg.time(args.c5_steps, 1)
        out = {"workload": wl.name + ": " + wl.notes, "steps": args.c5_steps, "warmup": 1,
               "encode_ms": round(sec * 1e3, 3), "comparisons_per_s": leg.triples / sec,
               "comparisons_per_step": leg.triples, "exhaustive_comparisons_per_step": leg.exhaustive,
               "dtype": leg.dtype(), "engine": leg.engine_desc(), "tiles": leg.tiles, "autotuned": False,
               "levels": leg.levels_json(), "stage_ms_per_step": leg.stage_ms(), "roofline": leg.roofline(),
               "decode": leg.decode(wl.decode_iters)}
    finally:
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed encodes (default: as many as fill about 5 s, at least 10)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_1024")
    ap.add_argument("--engine", default="mfma", choices=["mfma", "mfma_i8", "mfma_f16", "mfma_f16_16x16"],
                    help="matrix engine of the timed steps (mfma = the faster form per block size)")
    ap.add_argument("--pool-key", default="entropy", choices=["entropy", "variance"],
                    help="domain pool key: entropy (the paper's) or variance (the cited alternative)")
    ap.add_argument("--decode-iters", type=int, default=None,
                    help="decode each image after the timed encodes and report PSNR (default: the workload's)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each encode as a captured HIP graph (stage times then come from extra eager steps)")
    ap.add_argument("--fp32-steps", type=int, default=2, help="timed steps of the plain FP32 engine (0 skips)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in default tile shapes instead of running the autotuner first")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle sample budget (0 skips)")
    ap.add_argument("--c5-steps", type=int, default=5,
                    help="timed encodes of the 4096 x 4096 leg (0 skips it; skipped when it is the main workload)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 1 GiB device copy (HBM counter calibration for profiling runs)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this encoder build measures one GPU only; --gpus %d is not supported" % args.gpus)
        sys.exit(2)

    import torch

    from paper_1502_00324_amd import fic
    from paper_1502_00324_amd.configs import WORKLOADS
    from paper_1502_00324_amd.synth import sha256

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    ctx = fic.Context(0)
    pool_key = fic.POOL_VARIANCE if args.pool_key == "variance" else fic.POOL_ENTROPY
    engine = {"mfma": fic.ENGINE_MFMA, "mfma_i8": fic.ENGINE_MFMA_I8, "mfma_f16": fic.ENGINE_MFMA_F16,
              "mfma_f16_16x16": fic.ENGINE_MFMA_F16_16X16}[args.engine]
    leg = Leg(ctx, wl, engine, pool_key, dev, fic, torch)
    # the bytes recorded in the input manifest (same generator draws here)
    with open(os.path.join(ROOT, "tests", "golden", "synth_manifest.json")) as f:
        manifest = json.load(f).get(args.workload, [])
    inputs_match = [e["sha256"] for e in manifest] == [sha256(im) for im in leg.images]
    # tile shapes: the library's autotuner times every compiled shape of each
    # matrix level on these images (untimed here) and keeps the fastest
    leg.tune(not args.no_autotune)
    sec = leg.time(args.steps, args.warmup, args.graphs)
    value = leg.triples / sec
    roofline = leg.roofline()

    # the codec's output size (Sec. 3.3, Fig 7): pack every image once, untimed
    bits = {"header_bits": 0, "pool_bits": 0, "record_bits": 0, "total_bits": 0}
    for (pools, codes), im in zip(leg.bufs, leg.images):
        _, sz = ctx.pack(leg.p, im.shape[1], im.shape[0], pools, codes)
        for k in bits:
            bits[k] += sz[k]
    px = sum(im.size for im in leg.images)
    bitstream = {"bpp": round(bits["total_bits"] / px, 4), "cr": round(8.0 * px / bits["total_bits"], 3),
                 "bpp_codes_only": round(bits["record_bits"] / px, 4),
                 "cr_codes_only": round(8.0 * px / max(1, bits["record_bits"]), 3), **bits}

    # decode (Sec. 1-2) and PSNR (Eq 4), untimed by the step clock
    iters = wl.decode_iters if args.decode_iters is None else args.decode_iters
    decode = leg.decode(iters) if iters > 0 else None

    fp32 = None
    if args.fp32_steps > 0:
        pf = leg.mk(fic.ENGINE_FP32)
        bf = ctx.alloc_encode(leg.shapes(), pf, dev)
        ctx.encode(leg.imgs, pf, bf)
        ctx.set_timing(True)
        sec_f = run_steps(ctx, leg.imgs, pf, bf, args.fp32_steps, torch)
        st_f = ctx.read_timing()
        ctx.set_timing(False)
        fsearch = {B: v[0] / max(args.fp32_steps, 1) for (name, B), v in st_f.items() if name == "search"}
        msearch = {B: v[0] / max(leg.steps, 1) for (name, B), v in leg.stages.items() if name == "search"}
        fp32 = {"value": leg.triples / sec_f, "ms_per_step": round(sec_f * 1e3, 3),
                "speedup_mfma": round(sec_f / sec, 2),
                "search_ms_per_step": {str(B): round(v, 3) for B, v in fsearch.items()},
                "search_speedup_mfma": {str(B): round(fsearch[B] / msearch[B], 2) for B in fsearch if B in msearch},
                "codes_identical": same_outputs(leg.bufs, bf, leg.p.levels),
                "compared": "every level's codes (%s) and pools (%s)" % (", ".join(CODE_FIELDS),
                                                                         ", ".join(POOL_FIELDS))}
        del bf

    if args.copy_calib:
        # an elementwise kernel (not a DMA copy), so the counters see 1 GiB read + 1 GiB written
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 3, out=b)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": "range x domain x isometry comparisons/s (ranges searched, whole encode, all quadtree levels)",
        "value": value, "unit": "comparisons/s", "n_gpus": 1, "steps": leg.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3), "encode_ms_per_image": round(sec * 1e3 / len(leg.images), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": leg.dtype(),
        "data": "synthetic (seeded 1/f^2 noise + rectangles)",
        "inputs_match_manifest": inputs_match,
        "config": {"workload": wl.name + ": " + wl.notes, "images": len(leg.images),
                   "levels": [{"B": B, "L": L} for (B, L) in wl.levels],
                   "pool": "drop ceil(%d/%d * Nd) lowest-%s candidates" % (wl.pct + (args.pool_key,)),
                   "s_set": "k/16, k=0..16" if wl.s_den == 16 else "%s / %s" % (wl.s_num, wl.s_den),
                   "pool_max": wl.pool_max, "split_rms": wl.split_rms[0],
                   "engine": args.engine + ": " + leg.engine_desc(),
                   "parallelism": "single GPU", "graph_replay": bool(args.graphs),
                   "tiles": leg.tiles, "autotuned": not args.no_autotune},
        "comparisons_per_step": leg.triples,
        "exhaustive_comparisons_per_step": leg.exhaustive,
        "levels": leg.levels_json(),
        "stage_ms_per_step": leg.stage_ms(),
        "roofline": roofline, "fp32_baseline": fp32, "bitstream": bitstream, "decode": decode,
        "kernel_source_hash": kernel_source_hash(),
    }
    counts, images = leg.counts, leg.images
    del leg
    ctx.close()
    torch.cuda.empty_cache()
    if args.c5_steps > 0 and wl.name != "c5_4096":
        out["c5_4096"] = second_leg(fic, torch, dev, args)
        torch.cuda.empty_cache()
    # the oracle last: host work only, after every GPU leg
    out["cpu_baseline"] = cpu_baseline(wl, images, counts, args.cpu_seconds) if args.cpu_seconds > 0 else None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
