"""Runs libfic.so's host logic against the stub HIP runtime (started by
tests/test_host_logic.py with LD_LIBRARY_PATH pointing at the stub).

Every batched launch is checked against the per-kind workgroup prefix table
that the library uploaded for it: the grid must cover exactly the planned
workgroups, the prefixes must be non-decreasing, and each image's share of
the MFMA search must start on a multiple of 8 workgroups (the XCD mapping
relies on it).  Prints one JSON object with the results of each scenario.
"""
import ctypes
import json
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1502_00324_amd import fic  # noqa: E402
from paper_1502_00324_amd.synth import make_image  # noqa: E402

(K_LEVEL0, K_KEYS, K_HIST, K_PCMP, K_MOM, K_RANGE, K_AFRAG, K_BFRAG, K_VIEWS, K_DOMS, K_SEARCH, K_FINAL, K_CCMP,
 K_IROW, K_ICOL, K_ICSCAN) = range(16)
KIND_OF = [("k_level0", K_LEVEL0), ("k_pool_keys", K_KEYS), ("k_sel_hist", K_HIST), ("k_pool_moments", K_MOM),
           ("k_range_info", K_RANGE), ("k_mfma_afrag", K_AFRAG), ("k_mfma_bfrag", K_BFRAG),
           ("k_f16_afrag", K_AFRAG), ("k_f16_bfrag", K_BFRAG),
           ("k_fp32_views", K_VIEWS), ("k_fp32_doms", K_DOMS), ("k_mfma_search", K_SEARCH),
           ("k_f16_search", K_SEARCH), ("k_fp32_search", K_SEARCH), ("k_finalize", K_FINAL),
           ("k_integ_rows", K_IROW), ("k_integ_colsum", K_ICOL), ("k_integ_coladd", K_ICOL),
           ("k_integ_colscan", K_ICSCAN)]
PER_IMAGE = ("k_sel_init", "k_sel_pick", "k_bscan", "k_sel_fused")
ONE_BLOCK = ("k_search_plan",)
KIND_ARG = ("k_bcount", "k_bscatter")
NUM_KINDS = 16


class BatchDev(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("pre", ctypes.POINTER(ctypes.c_int32)), ("n", ctypes.c_int32),
                ("queue", ctypes.c_void_p)]


# resident workgroups of a persistent search under the stub: 2 per CU x 256 CUs
PERSISTENT_CAP = 512


HOOK = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_uint, ctypes.c_uint, ctypes.POINTER(ctypes.c_void_p))
log = {"launches": [], "errors": [], "forms": [], "shapes": []}


def on_launch(name, grid, block, args):
    name = name.decode()
    if "k_f16_prep" in name or "k_mfma_prep" in name:   # both operand builders in one launch
        bd = ctypes.cast(args[0], ctypes.POINTER(BatchDev)).contents
        n = bd.n
        pre = np.ctypeslib.as_array(bd.pre, shape=(NUM_KINDS * (n + 1),)).reshape(NUM_KINDS, n + 1).copy()
        na = ctypes.cast(args[1], ctypes.POINTER(ctypes.c_int32)).contents.value
        if na != pre[K_AFRAG, n] or grid != pre[K_AFRAG, n] + pre[K_BFRAG, n]:
            log["errors"].append("%s: grid %d (%d range blocks), planned %d + %d" % (name, grid, na, pre[K_AFRAG, n],
                                                                                   pre[K_BFRAG, n]))
        log["launches"].append(("k_prep", grid, None))
        return
    short = next((k for k, _ in KIND_OF if k in name), None) or next(
        (k for k in PER_IMAGE + KIND_ARG + ONE_BLOCK if k in name), None)
    if short is None:
        # kernels with no planned grid: logged by their short name
        m = re.match(r"_ZN3fic(\d+)", name)
        short = name[m.end():m.end() + int(m.group(1))] if m else name
        log["launches"].append((short, grid, None))
        return
    bd = ctypes.cast(args[0], ctypes.POINTER(BatchDev)).contents
    n = bd.n
    pre = np.ctypeslib.as_array(bd.pre, shape=(NUM_KINDS * (n + 1),)).reshape(NUM_KINDS, n + 1).copy()
    if (np.diff(pre, axis=1) < 0).any() or (pre[:, 0] != 0).any():
        log["errors"].append("%s: prefix table not a prefix sum" % short)
    if short in PER_IMAGE:
        want, kind = n, None
    elif short in ONE_BLOCK:
        want, kind = 1, None
    elif short in KIND_ARG:
        kind = ctypes.cast(args[1], ctypes.POINTER(ctypes.c_int32)).contents.value
        want = pre[kind, n]
    else:
        kind = dict(KIND_OF)[short]
        want = pre[kind, n]
        if short == "k_finalize":
            want = max(1, want)
        if short == "k_mfma_search":
            # operand form: the second template argument of the mangled name
            m = re.search(r"k_mfma_searchILi(\d+)ELi(\d+)E", name)
            log["forms"].append(int(m.group(2)) if m else -1)
        if short in ("k_mfma_search", "k_f16_search"):
            # the tile shape: (pl, rq, dt, wpe), pl = 0 for the 32x32 kernel
            a = [int(v) for v in re.findall(r"Li(\d+)E", name.split(short, 1)[1].split("EEv", 1)[0])]
            log["shapes"].append(a[1:] if short == "k_mfma_search" else [0] + a[1:])
        if short in ("k_mfma_search", "k_f16_search"):
            if (pre[kind] % 8 != 0).any():
                log["errors"].append("%s: an image's workgroups do not start on a multiple of 8" % short)
            # persistent: the resident workgroups, at most the static count
            want = min(want, PERSISTENT_CAP)
            if bd.queue is None:
                log["errors"].append("%s: no work queue" % short)
    if grid != want:
        log["errors"].append("%s: grid %d, planned %d" % (short, grid, want))
    log["launches"].append((short, grid, kind))


def buffers(keep, shape_caps):
    P, R = shape_caps

    def buf(m, dt):
        a = np.zeros(max(m, 1), dt)
        keep.append(a)
        return a.ctypes.data

    cnt = np.zeros(1, np.int32)
    keep.append(cnt)
    pool = fic.PoolC(P, buf(1, np.int32), buf(P, np.uint32), buf(P, np.int64), buf(P, np.uint32), buf(P, np.int64))
    codes = fic.CodesC(R, cnt.ctypes.data, buf(R, np.uint32), buf(R, np.uint8), buf(R, np.uint32), buf(R, np.uint8),
                       buf(R, np.uint8), buf(R, np.uint8), buf(R, np.int64))
    return pool, codes, cnt


def encode_case(L, h, shapes, levels, engine, pool_max=0, reps=2, timing_toggle=False, autotune=None):
    keep = []
    images = [make_image(11 + i, w, hh, 8) for i, (w, hh) in enumerate(shapes)]
    keep += images
    p = fic.make_params(levels, pool_max=pool_max, engine=engine)
    n, NL = len(images), p.levels
    imgs = (fic.Image * max(n, 1))(*[fic.Image(im.ctypes.data, im.shape[1], im.shape[0], im.shape[1])
                                     for im in images])
    pools = (fic.PoolC * max(n * NL, 1))()
    codes = (fic.CodesC * max(n * NL, 1))()
    for i, im in enumerate(images):
        pc = np.zeros(4, np.int64)
        rc = np.zeros(4, np.int64)
        L.fic_query_capacity(ctypes.byref(p), im.shape[1], im.shape[0], pc.ctypes.data, rc.ctypes.data)
        for l in range(NL):
            pools[i * NL + l], codes[i * NL + l], cnt = buffers(keep, (int(pc[l]), int(rc[l])))
            cnt[0] = int(rc[l])     # the kernels do not run: pretend every range splits
    statuses = []
    if autotune is not None:
        t = fic.Tuning()
        statuses.append(L.fic_autotune(h, imgs, n, ctypes.byref(p), pools, codes, 1, None, ctypes.byref(t)))
        autotune.update({"%d,%d" % (f, 1 << l): t.choice[f][l] for f in range(fic.FORMS) for l in range(6)
                         if t.choice[f][l] >= 0})
        return statuses
    for r in range(reps):
        if timing_toggle:
            L.fic_ctx_set_timing(h, 1)
        statuses.append(L.fic_encode(h, imgs, n, ctypes.byref(p), pools, codes, None))
        if timing_toggle:
            t = fic.Timing()
            statuses.append(L.fic_ctx_read_timing(h, ctypes.byref(t)))
            L.fic_ctx_set_timing(h, 0)
    return statuses


def main():
    L = fic.lib()
    hook = HOOK(on_launch)
    L.mock_set_hook(hook)
    L.mock_launches.restype = ctypes.c_long
    h = ctypes.c_void_p()
    assert L.fic_ctx_create(ctypes.byref(h), 0) == 0
    out = {}

    def scenario(name, fn):
        log["launches"], log["errors"], log["forms"], log["shapes"] = [], [], [], []
        st = fn()
        out[name] = {"status": st, "errors": list(log["errors"]), "launches": list(log["launches"]),
                     "forms": list(log["forms"]), "shapes": list(log["shapes"])}

    M, F, I8, H = fic.ENGINE_MFMA, fic.ENGINE_FP32, fic.ENGINE_MFMA_I8, fic.ENGINE_MFMA_F16
    X = fic.ENGINE_MFMA_F16_16X16
    mixed = [(128, 128), (256, 128), (64, 128), (1024, 512), (96, 96), (512, 512), (32, 32), (208, 144)]
    scenario("single_mfma", lambda: encode_case(L, h, [(64, 64)], [(8, 1), (4, 1)], M))
    scenario("single_fp32", lambda: encode_case(L, h, [(64, 64)], [(8, 1), (4, 1)], F))
    scenario("mixed_mfma_3lv", lambda: encode_case(L, h, mixed, [(16, 2), (8, 2), (4, 2)], M))
    scenario("mixed_fp32_3lv", lambda: encode_case(L, h, mixed, [(16, 2), (8, 2), (4, 2)], F))
    scenario("mixed_i8_3lv", lambda: encode_case(L, h, mixed, [(16, 2), (8, 2), (4, 2)], I8))
    scenario("mixed_f16_3lv", lambda: encode_case(L, h, mixed, [(16, 2), (8, 2), (4, 2)], H))
    scenario("mixed_f16x_3lv", lambda: encode_case(L, h, mixed, [(16, 2), (8, 2), (4, 2)], X))
    scenario("mixed_b32_4lv", lambda: encode_case(L, h, [(256, 256), (128, 64), (64, 64)],
                                                  [(32, 4), (16, 4), (8, 4), (4, 4)], M))
    scenario("paper_b2_cap", lambda: encode_case(L, h, [(64, 64), (32, 48)], [(16, 4), (8, 4), (4, 4), (2, 4)], M,
                                                 pool_max=64))
    scenario("min_images", lambda: encode_case(L, h, [(8, 8), (16, 8)], [(4, 1)], M))
    # more candidates than the one-workgroup selection takes: multi-block passes
    scenario("large_uncapped", lambda: encode_case(L, h, [(512, 512)], [(4, 1)], M, reps=1))
    scenario("large_capped", lambda: encode_case(L, h, [(512, 512)], [(4, 1)], M, pool_max=100, reps=1))
    scenario("timing_toggle", lambda: encode_case(L, h, mixed[:3], [(16, 2), (8, 2)], M, reps=3,
                                                  timing_toggle=True))
    scenario("empty_batch", lambda: encode_case(L, h, [], [(8, 1), (4, 1)], M))
    # graph replay: the first encode of a given argument set is captured, the
    # repeats launch nothing but the graph
    L.mock_captured.restype = L.mock_replays.restype = ctypes.c_long

    def graphs():
        L.fic_ctx_set_graphs(h, 2)
        c0, r0 = L.mock_captured(), L.mock_replays()
        st = encode_case(L, h, mixed[:3], [(16, 2), (8, 2), (4, 2)], M, reps=3)
        n1 = L.fic_ctx_graph_count(h)
        c1, r1, k1 = L.mock_captured(), L.mock_replays(), len(log["launches"])
        # a second argument set, then a third that evicts the least recently used
        st += encode_case(L, h, [(64, 64)], [(8, 1), (4, 1)], M, reps=1)
        st += encode_case(L, h, [(128, 64)], [(8, 1), (4, 1)], M, reps=1)
        n3 = L.fic_ctx_graph_count(h)
        L.fic_ctx_set_graphs(h, 0)
        n0 = L.fic_ctx_graph_count(h)
        log["graph"] = {"first_launches": k1, "first_captured": c1 - c0, "first_replays": r1 - r0,
                        "captured": L.mock_captured() - c0, "replays": L.mock_replays() - r0,
                        "counts": [n1, n3, n0]}
        return st

    scenario("graphs", graphs)
    out["graphs"]["graph"] = log["graph"]
    # tile shapes: the compiled candidates, the autotuner (all inert timings tie,
    # so the first candidate wins), and a forced choice
    cands = {}
    for f in range(fic.FORMS):
        for B in (2, 4, 8, 16, 32):
            cands["%d,%d" % (f, B)] = [list(fic.shape_describe(f, B, i)) for i in range(fic.shape_count(f, B))]
    out["candidates"] = cands
    for eng, name in ((I8, "i8"), (X, "f16x"), (H, "f16")):
        for B, Ls in ((32, 4), (16, 2), (8, 2), (4, 2), (2, 2)):
            if fic.level_engine(eng, B) == F:
                continue
            res = {}
            scenario("autotune_%s_%d" % (name, B),
                     lambda: encode_case(L, h, [(128, 128), (96, 64)], [(B, Ls)], eng, autotune=res))
            out["autotune_%s_%d" % (name, B)]["tuning"] = res

    def forced():
        t = fic.Tuning()
        L.fic_ctx_get_tuning(h, ctypes.byref(t))
        before = [list(r) for r in t.choice]
        t.choice[fic.FORM_I8][4] = 2        # B = 16: third candidate
        t.choice[fic.FORM_I8][3] = 1        # B = 8: second
        st = [L.fic_ctx_set_tuning(h, ctypes.byref(t))]
        bad = fic.Tuning()
        L.fic_ctx_get_tuning(h, ctypes.byref(bad))
        bad.choice[fic.FORM_I8][4] = 99
        log["bad_set"] = L.fic_ctx_set_tuning(h, ctypes.byref(bad))
        L.fic_ctx_get_tuning(h, ctypes.byref(bad))
        log["after_bad"] = [list(r) for r in bad.choice]
        log["before"] = before
        st += encode_case(L, h, [(128, 128)], [(16, 2), (8, 2), (4, 2)], I8, reps=1)
        for r in range(fic.FORMS):
            for l in range(6):
                t.choice[r][l] = -1
        st.append(L.fic_ctx_set_tuning(h, ctypes.byref(t)))
        return st

    scenario("tuning_forced", forced)
    out["tuning_forced"].update({k: log[k] for k in ("bad_set", "after_bad", "before")})
    # the allocation-free decoder: launches its kernels, allocates nothing
    # (timing on, so the ordinary decoder would create events), and refuses
    # an image above its fixed scratch before launching anything
    L.mock_allocs.restype = ctypes.c_long

    def decode_noalloc():
        keep = []
        p = fic.make_params([(8, 1), (4, 1)])
        W = H = 64
        pc, rc = np.zeros(4, np.int64), np.zeros(4, np.int64)
        L.fic_query_capacity(ctypes.byref(p), W, H, pc.ctypes.data, rc.ctypes.data)
        pools, codes = (fic.PoolC * 2)(), (fic.CodesC * 2)()
        for l in range(2):
            pools[l], codes[l], _ = buffers(keep, (int(pc[l]), int(rc[l])))
        out = np.zeros((H, W), np.uint8)
        L.fic_ctx_set_timing(h, 1)
        a0, k0 = L.mock_allocs(), len(log["launches"])
        st = [L.fic_decode_noalloc(h, ctypes.byref(p), pools, codes, W, H, 5, out.ctypes.data, None)]
        a1, k1 = L.mock_allocs(), len(log["launches"])
        st.append(L.fic_decode_noalloc(h, ctypes.byref(p), pools, codes, 8192, 4096, 5, out.ctypes.data, None))
        a2, k2 = L.mock_allocs(), len(log["launches"])
        st.append(L.fic_decode(h, ctypes.byref(p), pools, codes, W, H, 5, out.ctypes.data, None))
        a3 = L.mock_allocs()
        L.fic_ctx_set_timing(h, 0)
        log["noalloc"] = {"allocs": a1 - a0, "launches": k1 - k0, "over_allocs": a2 - a1,
                          "over_launches": k2 - k1, "decode_allocs": a3 - a2}
        return st

    scenario("decode_noalloc", decode_noalloc)
    out["decode_noalloc"]["noalloc"] = log["noalloc"]
    L.fic_ctx_set_scratch_limit(h, 1 << 10)
    scenario("over_limit", lambda: encode_case(L, h, [(1024, 1024)], [(8, 1), (4, 1)], M, reps=1))
    L.fic_ctx_set_scratch_limit(h, 0)
    L.fic_ctx_destroy(h)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
