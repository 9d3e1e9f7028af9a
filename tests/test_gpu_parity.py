"""Parity of the HIP encoder and decoder with the oracle, element by element:
pools (xy, key, sum4, A), codes (range xy, split, domain, isometry, s index,
offset, val_q), the child lists and the decoded image, for every search
engine (default MFMA mix, plain FP32, int8 MFMA, f16 MFMA).  Inputs are seeded synthetic images (paper_1502_00324_amd.synth)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1502_00324_amd import fic
from paper_1502_00324_amd.configs import WORKLOADS, K16
from paper_1502_00324_amd.synth import make_image

pytestmark = pytest.mark.gpu
WORKERS = max(1, min(16, os.cpu_count() or 1))
ENGINES = [fic.ENGINE_MFMA, fic.ENGINE_FP32, fic.ENGINE_MFMA_I8, fic.ENGINE_MFMA_F16, fic.ENGINE_MFMA_F16_16X16]
ENGINE_IDS = ["mfma", "fp32", "mfma_i8", "mfma_f16", "mfma_f16_16x16"]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    c = fic.Context(0)
    yield c
    c.close()


def params(levels, pct, pool_max, s_num, s_den, rms, engine):
    return fic.make_params(levels, pct=pct, pool_max=pool_max, s_num=s_num, s_den=s_den, split_rms=rms,
                           engine=engine)


def gpu_run(ctx, img, p, iters=None):
    H, W = img.shape
    t = torch.from_numpy(img).cuda()
    pools, codes = ctx.encode([t], p)[0]
    dec = ctx.decode(p, pools, codes, W, H, iters) if iters is not None else None
    torch.cuda.synchronize()
    return fic.levels_numpy(pools, codes, p), (dec.cpu().numpy() if dec is not None else None)


def oracle_run(img, levels, pct, pool_max, s_num, s_den, rms):
    return oracle.encode(img, levels, pct=pct, pool_max=pool_max, s_num=s_num, s_den=s_den, split_rms=rms,
                         workers=WORKERS)


def assert_levels_equal(got, ref, tag=""):
    assert len(got) == len(ref)
    for l, (g, r) in enumerate(zip(got, ref)):
        for f in ("xy", "key", "sum4", "a"):
            np.testing.assert_array_equal(g["pool"][f], r["pool"][f], err_msg="%s level %d pool %s" % (tag, l, f))
        np.testing.assert_array_equal(g["codes"]["xy"], r["ranges"], err_msg="%s level %d ranges" % (tag, l))
        for f in ("split", "domain", "iso", "s_idx", "offset", "err"):
            np.testing.assert_array_equal(g["codes"][f], r["codes"][f], err_msg="%s level %d %s" % (tag, l, f))


def gradient_energy(img, B0):
    """Per level-0 range: the sum of squared neighbour differences, the ranges
    most likely to split down to the last level."""
    H, W = img.shape
    f = img.astype(np.int64)
    ge = np.zeros_like(f)
    ge[:, :-1] += (f[:, 1:] - f[:, :-1]) ** 2
    ge[:-1, :] += (f[1:, :] - f[:-1, :]) ** 2
    return ge.reshape(H // B0, B0, W // B0, B0).sum(axis=(1, 3)).ravel()


def oracle_subtrees(img, pools, levels, ranges, s_num, s_den, rms):
    """The oracle's codes of the given level-0 ranges and their whole quadtree
    subtrees (Sec. 2, Fig 1), against the full pools: [(ranges, codes)] per level."""
    refs = []
    for l, (B, L) in enumerate(levels):
        last = l == len(levels) - 1
        ref = oracle.encode_level(img, pools[l]["xy"], ranges, B, list(s_num), s_den, rms, last, workers=WORKERS)
        refs.append((ranges, ref))
        if last:
            break
        ranges = oracle.children(ranges, ref["split"], B)
        if len(ranges) == 0:
            break
    return refs


def assert_pools_equal(got, pools, tag):
    for l, ref_pool in enumerate(pools):
        for f in ("xy", "key", "sum4", "a"):
            np.testing.assert_array_equal(got[l]["pool"][f], ref_pool[f], err_msg="%s level %d pool %s" % (tag, l, f))


def assert_subtrees_equal(got, refs, tag):
    """The GPU codes of the sampled ranges (found by position) equal the oracle's."""
    for l, (ranges, ref) in enumerate(refs):
        pos = {int(v): i for i, v in enumerate(got[l]["codes"]["xy"])}
        idx = np.array([pos[int(v)] for v in ranges], np.int64)
        for f in ("split", "domain", "iso", "s_idx", "offset", "err"):
            np.testing.assert_array_equal(got[l]["codes"][f][idx], ref[f], err_msg="%s level %d %s" % (tag, l, f))


def as_oracle_levels(got):
    """GPU codes and pools of one image in the oracle's level layout, so that
    the oracle decoder can rebuild an image from the GPU's own codes."""
    return [{"B": g["B"], "ranges": g["codes"]["xy"], "pool": g["pool"], "codes": g["codes"],
             "s_num": g["s_num"], "s_den": g["s_den"]} for g in got]


CASES = [
    # name, seed, W, H, n_rect, levels, pct, pool_max, s_num, s_den, split_rms
    ("c1_64", 0, 64, 64, 10, [(8, 4), (4, 4)], (3, 10), 0, K16, 16, (8, 1)),
    ("ragged_160x96", 1, 160, 96, 6, [(8, 4), (4, 4)], (3, 10), 0, K16, 16, (8, 1)),
    ("three_levels_L2", 2, 128, 64, 8, [(16, 2), (8, 2), (4, 2)], (3, 10), 0, K16, 16, (6, 1)),
    ("b4_L1_to_b2", 3, 64, 48, 4, [(4, 1), (2, 1)], (1, 2), 0, K16, 16, (8, 1)),
    ("paper_schedule_dn32", 4, 128, 128, 12, [(16, 4), (8, 4), (4, 4), (2, 4)], (0, 1), 32,
     ((1,), (2, 4), (3, 8), (5, 9)), 10, (8, 1)),
    ("all_split", 5, 64, 64, 2, [(8, 2), (4, 2)], (3, 10), 0, K16, 16, (0, 1)),
    ("none_split", 6, 64, 64, 2, [(8, 2), (4, 2)], (3, 10), 0, K16, 16, (255, 1)),
    ("b16_single_level", 7, 96, 96, 5, [(16, 2)], (3, 10), 0, K16, 16, (8, 1)),
    ("pct0_full_pool", 8, 64, 64, 5, [(8, 2), (4, 2)], (0, 1), 0, K16, 16, (5, 1)),
    ("odd_s_set", 9, 64, 64, 5, [(8, 4), (4, 4)], (3, 10), 0, (0, 3, 7, 10), 10, (7, 2)),
    # clustered contrasts: the search's start, taken from the line through the
    # end values, lands several steps from the chosen index
    ("clustered_s_set", 16, 96, 64, 8, [(8, 2), (4, 2)], (1, 10), 0, (0, 1, 2, 3, 4, 12, 14, 15, 16), 16, (6, 1)),
    ("b32_to_b16", 10, 128, 128, 10, [(32, 4), (16, 4)], (1, 2), 0, K16, 16, (8, 1)),
    # B = 32 over ~200 domain tiles with a ragged last tile, 3 range groups
    ("b32_multi_tile", 13, 256, 192, 12, [(32, 2), (16, 2)], (1, 2), 0, K16, 16, (8, 1)),
    ("pool_max_ties", 11, 96, 64, 30, [(8, 2), (4, 2)], (1, 10), 100, K16, 16, (6, 1)),
    # many flat rectangles and no entropy filter: constant domains (A = 0) in
    # the pool at B = 4 and 2, searched with and without s = 0 in S (without
    # it, flat ranges are searched too; with it, pairs tie at s = 0)
    ("flat_domains_s_without_0", 14, 96, 64, 40, [(4, 2), (2, 2)], (0, 1), 0, (1, 2, 3), 4, (4, 1)),
    ("flat_domains_k16", 15, 96, 64, 40, [(4, 1)], (0, 1), 0, K16, 16, (8, 1)),
]


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_encode_decode_parity(ctx, case, engine):
    name, seed, W, H, nrect, levels, pct, dn, s_num, s_den, rms = case
    print("case", name, "engine", engine, flush=True)
    img = make_image(seed, W, H, nrect)
    got, dec = gpu_run(ctx, img, params(levels, pct, dn, s_num, s_den, rms, engine), iters=6)
    ref = oracle_run(img, levels, pct, dn, s_num, s_den, rms)
    assert_levels_equal(got, ref, name)
    ref_dec = oracle.decode(W, H, ref, 6)
    np.testing.assert_array_equal(dec, ref_dec)
    assert oracle.psnr(img, dec) == oracle.psnr(img, ref_dec)


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_b32_extreme_magnitudes(ctx, engine):
    """Pixels 0 or 255 only: range and domain operands at their extremes, so
    the B = 32 cross term reaches the largest magnitudes the int32 planes
    hold (|C_hi| up to 2^24)."""
    rng = np.random.default_rng(5)
    img = (rng.integers(0, 2, (128, 160)) * 255).astype(np.uint8)
    levels = [(32, 2), (16, 2)]
    got, dec = gpu_run(ctx, img, params(levels, (1, 2), 0, K16, 16, (8, 1), engine), iters=4)
    ref = oracle_run(img, levels, (1, 2), 0, K16, 16, (8, 1))
    assert_levels_equal(got, ref, "b32_extreme")
    np.testing.assert_array_equal(dec, oracle.decode(160, 128, ref, 4))


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_small_blocks_extreme_magnitudes(ctx, engine):
    """Pixels 0 or 255 only at B = 4 and 2: the mean-centred operands of the
    one-step levels reach +-255 and +-1020, the cross terms their largest
    magnitudes, and most ranges split (S with 0 and 1 only keeps errors up)."""
    rng = np.random.default_rng(8)
    img = (rng.integers(0, 2, (48, 80)) * 255).astype(np.uint8)
    levels = [(4, 1), (2, 1)]
    for s_num, s_den in ((K16, 16), ((0, 1), 1)):
        got, dec = gpu_run(ctx, img, params(levels, (1, 4), 0, s_num, s_den, (20, 1), engine), iters=4)
        ref = oracle_run(img, levels, (1, 4), 0, list(s_num), s_den, (20, 1))
        assert_levels_equal(got, ref, "small_extreme")
        np.testing.assert_array_equal(dec, oracle.decode(80, 48, ref, 4))


@pytest.mark.parametrize("engine", [fic.ENGINE_MFMA, fic.ENGINE_FP32], ids=["mfma", "fp32"])
def test_b32_xcd_chunks(ctx, engine):
    """512 x 512 at B = 32, L = 2: ~25 k domains in ~40 chunks, enough for the
    XCD-aware chunk walk and the cross-workgroup best sharing."""
    img = make_image(14, 512, 512, 40)
    levels = [(32, 2)]
    got, _ = gpu_run(ctx, img, params(levels, (1, 2), 0, K16, 16, (8, 1), engine))
    ref = oracle_run(img, levels, (1, 2), 0, K16, 16, (8, 1))
    assert_levels_equal(got, ref, "b32_xcd")


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_constant_and_block_constant_images(ctx, engine):
    rng = np.random.default_rng(99)
    for img in (np.full((64, 64), 77, np.uint8),
                np.kron(rng.integers(0, 256, (8, 8)), np.ones((8, 8), np.int64)).astype(np.uint8)):
        p = params([(8, 4), (4, 4)], (3, 10), 0, K16, 16, (8, 1), engine)
        got, dec = gpu_run(ctx, img, p, iters=3)
        c = got[0]["codes"]
        assert (c["domain"] == 0).all() and (c["iso"] == 0).all() and (c["s_idx"] == 0).all()
        assert (c["err"] == 0).all() and (c["split"] == 0).all() and len(got[1]["codes"]["xy"]) == 0
        np.testing.assert_array_equal(dec, img)


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_tied_entropy_pool_larger_than_planned(ctx, engine):
    """Every 2B x 2B window of a period-2 pattern has the same histogram, so
    all entropy keys tie, the percentile drops nothing strictly and the
    equal-to-minimum rule keeps every candidate: the pool exceeds the size
    the chunks were planned for (Nd - ceil(p Nd)), and the searched ranges
    (not constant) must still see every domain."""
    yy, xx = np.mgrid[0:96, 0:128]
    for img in (np.where((yy + xx) % 2 == 0, 60, 190).astype(np.uint8),
                np.where(xx % 2 == 0, 30, 220).astype(np.uint8)):
        levels = [(8, 2), (4, 2)]
        p = params(levels, (3, 10), 0, K16, 16, (8, 1), engine)
        got, _ = gpu_run(ctx, img, p)
        ref = oracle_run(img, levels, (3, 10), 0, K16, 16, (8, 1))
        nd = ((128 - 16) // 2 + 1) * ((96 - 16) // 2 + 1)
        assert len(ref[0]["pool"]["xy"]) == nd
        assert_levels_equal(got, ref, "tied_pool")


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_config2_512_full_parity(ctx, engine):
    wl = WORKLOADS["c2_512"]
    seed, W, H, nrect = wl.images[0]
    img = make_image(seed, W, H, nrect)
    p = params(wl.levels, wl.pct, wl.pool_max, wl.s_num, wl.s_den, wl.split_rms, engine)
    got, dec = gpu_run(ctx, img, p, iters=8)
    ref = oracle_run(img, wl.levels, wl.pct, wl.pool_max, list(wl.s_num), wl.s_den, wl.split_rms)
    assert_levels_equal(got, ref, "c2")
    np.testing.assert_array_equal(dec, oracle.decode(W, H, ref, 8))


@pytest.fixture(scope="module")
def c3_reference():
    """Full-size c3 (L = 1, ~0.7 M domains per level): the oracle's pools in
    full and the codes of 24 seeded level-0 ranges with their whole quadtree
    subtrees."""
    wl = WORKLOADS["c3_1024"]
    seed, W, H, nrect = wl.images[0]
    img = make_image(seed, W, H, nrect)
    pools = [oracle.build_pool(img, B, L, wl.pct, wl.pool_max, threads=WORKERS) for (B, L) in wl.levels]
    all0 = oracle.level0_ranges(W, H, wl.levels[0][0])
    rng = np.random.default_rng(2024)
    ranges = all0[np.sort(rng.choice(len(all0), 24, replace=False))]
    refs = oracle_subtrees(img, pools, wl.levels, ranges, wl.s_num, wl.s_den, wl.split_rms)
    return wl, img, all0, pools, refs


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_config3_1024_sampled_parity(ctx, c3_reference, engine):
    """Every engine on the full-size c3 workload, in the launch configuration
    the benchmark times: both pools in full, the sampled subtrees exactly."""
    wl, img, all0, pools, refs = c3_reference
    print("c3 engine", engine, "subtree ranges per level", [len(r) for r, _ in refs], flush=True)
    p = params(wl.levels, wl.pct, wl.pool_max, wl.s_num, wl.s_den, wl.split_rms, engine)
    got, _ = gpu_run(ctx, img, p)
    assert_pools_equal(got, pools, "c3")
    np.testing.assert_array_equal(got[0]["codes"]["xy"], all0)
    assert_subtrees_equal(got, refs, "c3")


@pytest.fixture(scope="module")
def c5_reference():
    """Full-size c5 (4096^2, B 32 -> 16 -> 8 -> 4): the oracle's four pools in
    full (4.07 M to 16.7 M candidates) and the codes of 12 level-0 ranges with
    their whole quadtree subtrees.  Few level-0 ranges of this image split, so
    the sample is the 12 with the largest gradient energy (sum of squared
    neighbour differences), the ones most likely to reach the lower levels."""
    wl = WORKLOADS["c5_4096"]
    seed, W, H, nrect = wl.images[0]
    img = make_image(seed, W, H, nrect)
    pools = [oracle.build_pool(img, B, L, wl.pct, wl.pool_max, threads=WORKERS) for (B, L) in wl.levels]
    B0 = wl.levels[0][0]
    energy = gradient_energy(img, B0)
    all0 = oracle.level0_ranges(W, H, B0)
    ranges = all0[np.sort(np.argsort(-energy, kind="stable")[:12])]
    refs = oracle_subtrees(img, pools, wl.levels, ranges, wl.s_num, wl.s_den, wl.split_rms)
    return wl, img, all0, pools, refs


@pytest.mark.timeout(900)
@pytest.mark.parametrize("engine", [fic.ENGINE_MFMA, fic.ENGINE_FP32], ids=["mfma", "fp32"])
def test_config5_4096_sampled_parity(ctx, c5_reference, engine):
    """c5 in full size: pools in full, sampled subtrees exactly, and (matrix
    engine) the GPU's 8-iteration decode of its own codes equal to the
    oracle decoder's on the same leaves, with equal PSNR (Eq 4)."""
    wl, img, all0, pools, refs = c5_reference
    print("c5 engine", engine, "subtree ranges per level", [len(r) for r, _ in refs], flush=True)
    p = params(wl.levels, wl.pct, wl.pool_max, wl.s_num, wl.s_den, wl.split_rms, engine)
    iters = wl.decode_iters if engine == fic.ENGINE_MFMA else None
    got, dec = gpu_run(ctx, img, p, iters=iters)
    assert_pools_equal(got, pools, "c5")
    np.testing.assert_array_equal(got[0]["codes"]["xy"], all0)
    assert_subtrees_equal(got, refs, "c5")
    if iters:
        H, W = img.shape
        ref_dec = oracle.decode(W, H, as_oracle_levels(got), iters)
        np.testing.assert_array_equal(dec, ref_dec)
        assert oracle.psnr(img, dec) == oracle.psnr(img, ref_dec)
        print("c5 decode: %d iterations, PSNR %.3f dB" % (iters, oracle.psnr(img, dec)), flush=True)


@pytest.fixture(scope="module")
def c4_reference():
    """The c4 batch (64 images of uneven sizes, B 16 -> 8 -> 4, L = 2): every
    pool of every image in full from the oracle, and per image the codes of 5
    level-0 ranges with their whole subtrees (3 seeded at random, 2 of the
    largest gradient energy)."""
    wl = WORKLOADS["c4_batch64"]
    images = [make_image(s, w, h, n) for (s, w, h, n) in wl.images]
    B0 = wl.levels[0][0]
    out = []
    for i, img in enumerate(images):
        H, W = img.shape
        pools = [oracle.build_pool(img, B, L, wl.pct, wl.pool_max, threads=WORKERS) for (B, L) in wl.levels]
        all0 = oracle.level0_ranges(W, H, B0)
        rng = np.random.default_rng(400 + i)
        top = np.argsort(-gradient_energy(img, B0), kind="stable")[:2]
        rest = np.setdiff1d(np.arange(len(all0)), top)
        pick = np.sort(np.concatenate([top, rng.choice(rest, 3, replace=False)]))
        refs = oracle_subtrees(img, pools, wl.levels, all0[pick], wl.s_num, wl.s_den, wl.split_rms)
        out.append((all0, pools, refs))
    return wl, images, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
def test_config4_batch64_parity(ctx, c4_reference, engine):
    """The whole c4 batch in one fic_encode (one launch set per level over
    the 64 images, per-image prefix tables, shared scratch), image by image
    against the oracle: every pool in full, the level-0 range lists, and the
    sampled subtrees exactly."""
    wl, images, refs = c4_reference
    p = params(wl.levels, wl.pct, wl.pool_max, wl.s_num, wl.s_den, wl.split_rms, engine)
    batch = ctx.encode([torch.from_numpy(im).cuda() for im in images], p)
    torch.cuda.synchronize()
    deep = 0
    for i, ((pools, codes), (all0, ref_pools, sub)) in enumerate(zip(batch, refs)):
        got = fic.levels_numpy(pools, codes, p)
        tag = "c4 image %d (%dx%d)" % (i, images[i].shape[1], images[i].shape[0])
        assert_pools_equal(got, ref_pools, tag)
        np.testing.assert_array_equal(got[0]["codes"]["xy"], all0, err_msg=tag)
        assert_subtrees_equal(got, sub, tag)
        deep += len(sub) == len(wl.levels)
    print("c4 engine", engine, ": subtrees reaching the last level in", deep, "of 64 images", flush=True)
    assert deep > 0


def test_stepwise_entry_points_match_oracle(ctx):
    """fic_build_domain_pool + fic_encode_level driven one level at a time."""
    img = make_image(12, 96, 64, 8)
    levels = [(8, 2), (4, 2)]
    ref = oracle_run(img, levels, (3, 10), 0, K16, 16, (6, 1))
    t = torch.from_numpy(img).cuda()
    xy = torch.from_numpy(oracle.level0_ranges(96, 64, 8).view(np.int32)).cuda()
    n = torch.tensor([len(xy)], dtype=torch.int32, device="cuda")
    cap = len(xy)
    for l, (B, L) in enumerate(levels):
        pool = ctx.build_domain_pool(t, B, L, (3, 10), 0)
        last = l == len(levels) - 1
        codes, children, nch = ctx.encode_level(t, pool, xy, n, cap, B, K16, 16, (6, 1), last, fic.ENGINE_MFMA)
        torch.cuda.synchronize()
        g = codes.numpy()
        for f in ("split", "domain", "iso", "s_idx", "offset", "err"):
            np.testing.assert_array_equal(g[f], ref[l]["codes"][f], err_msg="level %d %s" % (l, f))
        np.testing.assert_array_equal(pool.numpy()["xy"], ref[l]["pool"]["xy"])
        if not last:
            xy, n, cap = children, nch, 4 * cap


def test_determinism_and_batch_independence(ctx):
    imgs = [make_image(s, w, h, 6) for s, w, h in [(20, 64, 64), (21, 128, 64), (22, 96, 96)]]
    p = params([(16, 2), (8, 2), (4, 2)], (3, 10), 0, K16, 16, (6, 1), fic.ENGINE_MFMA)
    batch = ctx.encode([torch.from_numpy(im).cuda() for im in imgs], p)
    torch.cuda.synchronize()
    for im, (pools, codes) in zip(imgs, batch):
        alone, _ = gpu_run(ctx, im, p)
        again, _ = gpu_run(ctx, im, p)
        together = fic.levels_numpy(pools, codes, p)
        ref = oracle_run(im, [(16, 2), (8, 2), (4, 2)], (3, 10), 0, K16, 16, (6, 1))
        assert_levels_equal(together, ref, "batched %dx%d" % (im.shape[1], im.shape[0]))
        for a, b, c in zip(alone, again, together):
            for f in ("split", "domain", "iso", "s_idx", "offset", "err", "xy"):
                np.testing.assert_array_equal(a["codes"][f], b["codes"][f])
                np.testing.assert_array_equal(a["codes"][f], c["codes"][f])


VARIANCE_CASES = [
    ("var_two_levels", 31, 96, 64, 8, [(8, 2), (4, 2)], (3, 10), 0, K16, 16, (6, 1)),
    ("var_paper_dn32", 32, 128, 128, 12, [(16, 4), (8, 4), (4, 4), (2, 4)], (0, 1), 32,
     ((1,), (2, 4), (3, 8), (5, 9)), 10, (8, 1)),
    ("var_b32", 33, 128, 128, 10, [(32, 4), (16, 4)], (1, 2), 0, K16, 16, (8, 1)),
]


# (B, L, pct, DN): steps below, at and above the window side 2B (the sliding
# and the reloading key update), odd steps, on an image of odd width and height
# (unaligned rows)
POOL_GEOMS = [(2, 1, (3, 10), 0), (2, 3, (1, 2), 0), (2, 5, (3, 10), 40), (4, 3, (3, 10), 0), (4, 9, (0, 1), 0),
              (8, 1, (3, 10), 0), (8, 7, (1, 2), 25), (16, 3, (3, 10), 0), (16, 33, (0, 1), 0), (32, 5, (3, 10), 0),
              (32, 70, (0, 1), 0)]


@pytest.mark.parametrize("geom", POOL_GEOMS, ids=lambda g: "B%d_L%d" % g[:2])
def test_entropy_pool_any_step(ctx, geom):
    """The entropy pool alone (Sec. 3, Eq 5-6) against the oracle: candidate
    keys of every window size, selection, compaction and moments."""
    B, L, pct, dn = geom
    W, H = 203, 139
    img = make_image(50 + B + L, W, H, 7)
    ref = oracle.build_pool(img, B, L, pct, dn)
    pool = ctx.build_domain_pool(torch.from_numpy(img).cuda(), B, L, pct, dn)
    torch.cuda.synchronize()
    got = pool.numpy()
    assert len(got["xy"]) == len(ref["xy"]) > 0
    for f in ("xy", "key", "sum4", "a"):
        np.testing.assert_array_equal(got[f], ref[f], err_msg=f)


@pytest.mark.parametrize("engine", [fic.ENGINE_MFMA, fic.ENGINE_FP32], ids=["mfma", "fp32"])
@pytest.mark.parametrize("case", VARIANCE_CASES, ids=lambda c: c[0])
def test_variance_pool_parity(ctx, case, engine):
    """The variance-keyed pool (the alternative cited in Sec. 1) through the
    whole encode: pools (xy, key, sum4, A) and codes equal the oracle's."""
    name, seed, W, H, nr, levels, pct, dn, s_num, s_den, rms = case
    img = make_image(seed, W, H, nr)
    p = fic.make_params(levels, pct=pct, pool_max=dn, s_num=s_num, s_den=s_den, split_rms=rms, engine=engine,
                        pool_key=fic.POOL_VARIANCE)
    got, _ = gpu_run(ctx, img, p)
    ref = oracle.encode(img, levels, pct=pct, pool_max=dn, s_num=s_num, s_den=s_den, split_rms=rms,
                        workers=WORKERS, pool_key="variance")
    assert_levels_equal(got, ref, name)


def test_graph_replay_matches_eager_encodes(ctx):
    """fic_ctx_set_graphs: the first encode of an argument set is captured,
    repeats are graph replays.  Each replay (with eager work and a
    synchronisation between replays, and a new image written in place) is
    compared with an eager encode of the same image in another context."""
    shapes = [(128, 64), (64, 64), (96, 96)]
    p = params([(16, 2), (8, 2), (4, 2)], (3, 10), 0, K16, 16, (6, 1), fic.ENGINE_MFMA)
    eager = fic.Context(0)
    g = fic.Context(0)
    g.set_graphs(4)
    host = [make_image(40 + i, w, h, 8) for i, (w, h) in enumerate(shapes)]
    host2 = [make_image(60 + i, w, h, 12) for i, (w, h) in enumerate(shapes)]
    lv = [(16, 2), (8, 2), (4, 2)]
    refs = {id(im): oracle_run(im, lv, (3, 10), 0, K16, 16, (6, 1)) for im in host + host2}
    imgs = [torch.from_numpy(im).cuda() for im in host]
    bufs = g.alloc_encode(shapes, p, imgs[0].device)
    try:
        for rep in range(4):
            if rep == 2:   # new contents at the same addresses
                for i in range(len(shapes)):
                    imgs[i].copy_(torch.from_numpy(host2[i]).cuda())
            cur = host if rep < 2 else host2
            g.encode(imgs, p, bufs)
            torch.cuda.synchronize()
            assert g.graph_count() == 1
            ref = eager.encode(imgs, p)
            junk = torch.randn(1 << 16, device=imgs[0].device).sum()   # eager work between replays
            torch.cuda.synchronize()
            del junk
            for (pools, codes), (rp, rc), im in zip(bufs, ref, cur):
                got = fic.levels_numpy(pools, codes, p)
                want = fic.levels_numpy(rp, rc, p)
                assert_levels_equal(got, refs[id(im)], "replay %d" % rep)
                for a, b in zip(got, want):
                    for f in ("xy", "split", "domain", "iso", "s_idx", "offset", "err"):
                        np.testing.assert_array_equal(a["codes"][f], b["codes"][f], err_msg="replay %d %s" % (rep, f))
                    for f in ("xy", "key", "sum4", "a"):
                        np.testing.assert_array_equal(a["pool"][f], b["pool"][f], err_msg="replay %d pool %s" % (rep, f))
        # a second argument set gets its own graph; the first still replays
        p2 = params([(8, 2), (4, 2)], (3, 10), 0, K16, 16, (8, 1), fic.ENGINE_MFMA)
        one = [imgs[1]]
        b2 = g.alloc_encode([shapes[1]], p2, imgs[0].device)
        g.encode(one, p2, b2)
        g.encode(imgs, p, bufs)
        torch.cuda.synchronize()
        assert g.graph_count() == 2
        ref2 = eager.encode(one, p2)
        torch.cuda.synchronize()
        for a, b in zip(fic.levels_numpy(*b2[0], p2), fic.levels_numpy(*ref2[0], p2)):
            np.testing.assert_array_equal(a["codes"]["domain"], b["codes"]["domain"])
            np.testing.assert_array_equal(a["codes"]["err"], b["codes"]["err"])
    finally:
        g.set_graphs(0)
        g.close()
        eager.close()


def test_failure_paths_return_status_without_launch(ctx):
    img = torch.from_numpy(make_image(30, 64, 64, 3)).cuda()
    p = params([(8, 4), (4, 4)], (3, 10), 0, K16, 16, (8, 1), fic.ENGINE_MFMA)
    (pools, codes), = ctx.alloc_encode([(64, 64)], p, img.device)
    small = fic.Pool.alloc(5, img.device)
    with pytest.raises(fic.FicError) as e:
        ctx.encode([img], p, bufs=[([small, pools[1]], codes)])
    assert e.value.status == fic.FIC_E_CAPACITY
    bad = params([(8, 4), (4, 4)], (3, 10), 0, K16, 16, (8, 1), fic.ENGINE_MFMA)
    bad.s_num[0][3] = 1   # not ascending
    with pytest.raises(fic.FicError) as e:
        ctx.encode([img], bad)
    assert e.value.status == fic.FIC_E_INVALID
    limited = fic.Context(0)
    limited.set_scratch_limit(1024)
    with pytest.raises(fic.FicError) as e:
        limited.encode([img], p)
    assert e.value.status == fic.FIC_E_NOMEM
    limited.close()
    # the shared context still works after the refused calls
    got, _ = gpu_run(ctx, make_image(0, 64, 64, 10), p)
    assert len(got[0]["codes"]["xy"]) == 64
