"""Pins for the oracle.

Every check here rests on something other than the oracle itself: the
paper's worked numbers (tests/golden), closed forms of Eq 4-6, numpy/scipy
library routines (decimation, rotations, entropy), exhaustive brute force of
Eq 1 per pixel (Fractions on the smallest case), special cases whose answer
is known by hand, and metamorphic relations (gray shift, gray inversion).
"""
import json
import math
import os
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

from paper_1502_00324_amd.synth import make_image

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
K16 = list(range(17))


def ref_decimate(block):
    """2x2 sums of a 2B x 2B block (numpy reshape)."""
    b = block.shape[0] // 2
    return block.astype(np.int64).reshape(b, 2, b, 2).sum(axis=(1, 3))


def ref_iso(block, t):
    """numpy reference of isometry t = 4m + r: r clockwise turns, then fliplr if m."""
    out = np.rot90(block, -(t & 3))
    return np.fliplr(out) if t >> 2 else out


def orc_iso(orc, block, t):
    B = block.shape[0]
    out = np.empty_like(block)
    for y in range(B):
        for x in range(B):
            sy, sx = orc.iso_source(t, B, y, x)
            out[y, x] = block[sy, sx]
    return out


def exact_entropy_rank_key(block):
    """prod q^q over the gray-level counts: an exact big integer that orders
    blocks of one size by entropy (larger product = lower entropy)."""
    out = 1
    for q in np.bincount(block.ravel(), minlength=256).tolist():
        if q > 1:
            out *= q ** q
    return out


def entropy_from_key(g, m):
    return math.log(m) - g / (m * 2.0 ** 32)


def float_entropy(block):
    """Eq 5-6 with scipy, summed over the sorted counts (canonical order)."""
    counts = np.sort(np.bincount(block.ravel(), minlength=256))
    counts = counts[counts > 0]
    return float(scipy.stats.entropy(counts))


# ---------------------------------------------------------------- candidates
def test_worked_examples_from_paper(orc):
    with open(os.path.join(GOLDEN, "paper_worked_examples.json")) as f:
        gold = json.load(f)
    ex = gold["domain_count_512_16_step4"]
    # 16 x 16 domains means range size B = 8
    assert len(orc.candidates(ex["image"], ex["image"], ex["domain"] // 2, ex["step"])) == ex["count"]


def test_candidate_count_full_step(orc):
    # (N - 2n + 1)^2 domains of size 2n at step 1 (Sec. 1)
    for N, n in [(64, 4), (40, 8), (33, 5)]:
        assert len(orc.candidates(N, N, n, 1)) == (N - 2 * n + 1) ** 2


def test_candidate_closed_form_and_raster_order(orc):
    W, H, B, L = 100, 60, 8, 3
    xy = orc.candidates(W, H, B, L)
    assert len(xy) == ((W - 2 * B) // L + 1) * ((H - 2 * B) // L + 1)
    ys, xs = (xy >> 16).astype(int), (xy & 0xFFFF).astype(int)
    assert (np.lexsort((xs, ys)) == np.arange(len(xy))).all()
    assert set(np.unique(xs)) == set(range(0, W - 2 * B + 1, L))
    assert set(np.unique(ys)) == set(range(0, H - 2 * B + 1, L))


def test_range_count(orc):
    # (N/n)^2 range blocks (Sec. 1)
    assert len(orc.level0_ranges(512, 512, 16)) == (512 // 16) ** 2


# ---------------------------------------------------------------- entropy
def test_entropy_table_regenerates():
    here = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "gen_entropy_table.py")
    assert subprocess.call([sys.executable, here, "--check"]) == 0


def test_entropy_table_vs_float_log(orc):
    T = orc.entropy_table()
    assert T[0] == 0 and T[1] == 0
    q = np.arange(2, 4097, dtype=np.float64)
    ref = q * np.log(q) * 2.0 ** 32
    # each of at most 12 prime logarithms is rounded to 2^-32
    assert (np.abs(T[2:].astype(np.float64) - ref) <= q * 6 + 1).all()
    # additivity: equal products prod q^q give equal keys
    assert T[4] + 4 * T[1] == 4 * T[2]
    assert T[8] == 12 * T[2] and T[12] == 12 * (T[4] // 4 + T[3] // 3)


def test_entropy_closed_forms(orc):
    m = 256
    flat = np.full((16, 16), 77, np.uint8)
    assert abs(entropy_from_key(orc.entropy_key(flat, 0, 0, 16), m)) < 1e-8
    halves = np.full((16, 16), 10, np.uint8)
    halves[8:] = 200
    assert abs(entropy_from_key(orc.entropy_key(halves, 0, 0, 16), m) - math.log(2)) < 1e-8
    rng = np.random.default_rng(3)
    every = rng.permutation(256).astype(np.uint8).reshape(16, 16)
    assert abs(entropy_from_key(orc.entropy_key(every, 0, 0, 16), m) - math.log(256)) < 1e-8


def test_entropy_random_blocks_vs_scipy(orc):
    img = make_image(5, 96, 96, 6)
    for (x, y, s) in [(0, 0, 8), (13, 40, 16), (50, 7, 32), (3, 3, 4), (60, 60, 24)]:
        blk = img[y:y + s, x:x + s]
        assert abs(entropy_from_key(orc.entropy_key(img, x, y, s), s * s) - float_entropy(blk)) < 1e-8


def test_entropy_key_keeps_exact_ties(orc):
    # counts {4,1,1,1,1} and {2,2,2,2}: both have sum q ln q = 8 ln 2
    a = np.array([[7, 7, 7, 7], [1, 2, 3, 4]], np.uint8)
    b = np.array([[9, 9, 5, 5], [6, 6, 8, 8]], np.uint8)
    wide_a = np.zeros((4, 4), np.uint8)
    wide_b = np.zeros((4, 4), np.uint8)
    wide_a[:2, :] = a
    wide_a[2:, :] = np.array([[10, 11, 12, 13], [14, 15, 16, 17]])
    wide_b[:2, :] = b
    wide_b[2:, :] = np.array([[10, 11, 12, 13], [14, 15, 16, 17]])
    assert exact_entropy_rank_key(wide_a) == exact_entropy_rank_key(wide_b)
    assert orc.entropy_key(wide_a, 0, 0, 4) == orc.entropy_key(wide_b, 0, 0, 4)


# ---------------------------------------------------------------- pool
def ref_pool(img, B, L, pct, pool_max=0):
    """Pool by exact entropy order (big-integer prod q^q): drop ceil(p*Nd)
    lowest-entropy candidates, keep those of strictly higher entropy."""
    H, W = img.shape
    cands = [(y, x) for y in range(0, H - 2 * B + 1, L) for x in range(0, W - 2 * B + 1, L)]
    key = [exact_entropy_rank_key(img[y:y + 2 * B, x:x + 2 * B]) for (y, x) in cands]
    nd = len(cands)
    c = -(-pct[0] * nd // pct[1])
    if c == 0:
        keep = [True] * nd
    else:
        thr = sorted(key, reverse=True)[c - 1]
        keep = [k < thr for k in key]
        if not any(keep):
            keep = [k == min(key) for k in key]
    idx = [i for i in range(nd) if keep[i]]
    if pool_max and len(idx) > pool_max:
        idx = sorted(sorted(idx, key=lambda i: (key[i], i))[:pool_max])
    return [cands[i] for i in idx]


@pytest.mark.parametrize("seed,W,H,B,L,pct,dn", [
    (0, 64, 64, 8, 4, (3, 10), 0),
    (1, 48, 40, 4, 2, (3, 10), 0),
    (2, 40, 40, 4, 1, (1, 2), 0),
    (3, 64, 48, 4, 4, (0, 1), 0),
    (4, 64, 64, 8, 4, (3, 10), 32),
    (5, 48, 48, 4, 2, (0, 1), 64),
])
def test_pool_matches_float_entropy_reference(orc, seed, W, H, B, L, pct, dn):
    img = make_image(seed, W, H, 4)
    pool = orc.build_pool(img, B, L, pct, dn)
    got = [(int(v >> 16), int(v & 0xFFFF)) for v in pool["xy"]]
    assert got == ref_pool(img, B, L, pct, dn)


def test_pool_p0_keeps_all(orc):
    img = make_image(7, 64, 64, 3)
    pool = orc.build_pool(img, 4, 2, (0, 1))
    assert (pool["xy"] == orc.candidates(64, 64, 4, 2)).all()


def test_pool_distinct_keys_size(orc):
    # with all candidate entropies distinct, the pool is exactly Nd - ceil(p Nd)
    cands = orc.candidates(64, 64, 8, 4)
    nd = len(cands)
    for seed in range(100):
        img = np.random.default_rng(seed).integers(0, 16, (64, 64)).astype(np.uint8)
        exact = {exact_entropy_rank_key(img[v >> 16:(v >> 16) + 16, v & 0xFFFF:(v & 0xFFFF) + 16]) for v in cands}
        if len(exact) == nd:
            break
    else:
        pytest.fail("no image with distinct entropies")
    keys = [orc.entropy_key(img, int(v & 0xFFFF), int(v >> 16), 16) for v in cands]
    assert len(set(keys)) == nd
    for pct in [(3, 10), (1, 2), (1, 3)]:
        c = -(-pct[0] * nd // pct[1])
        assert len(orc.build_pool(img, 8, 4, pct)["xy"]) == nd - c


def test_pool_ties_drop_whole_tie_class(orc):
    # left half flat (zero entropy), right half noise: every flat candidate ties
    rng = np.random.default_rng(12)
    img = np.full((32, 64), 90, np.uint8)
    img[:, 32:] = rng.integers(0, 256, (32, 32))
    cands = orc.candidates(64, 32, 4, 4)
    flat = np.array([(v & 0xFFFF) + 8 <= 32 for v in cands])
    pool = orc.build_pool(img, 4, 4, (1, 10))
    assert len(pool["xy"]) == int((~flat).sum())


def test_pool_empty_fallback_keeps_max_entropy(orc):
    img = np.full((32, 32), 5, np.uint8)
    pool = orc.build_pool(img, 4, 4, (3, 10))
    assert (pool["xy"] == orc.candidates(32, 32, 4, 4)).all()


def test_pool_moments_vs_numpy(orc):
    img = make_image(9, 64, 64, 5)
    B = 8
    pool = orc.build_pool(img, B, 4, (3, 10))
    n = B * B
    for v, s4, a in zip(pool["xy"], pool["sum4"], pool["a"]):
        x, y = int(v & 0xFFFF), int(v >> 16)
        d4 = ref_decimate(img[y:y + 2 * B, x:x + 2 * B])
        assert int(s4) == int(d4.sum())
        assert int(a) == n * int((d4 * d4).sum()) - int(d4.sum()) ** 2


# ---------------------------------------------------------------- isometries
@pytest.mark.parametrize("B", [2, 3, 4, 8])
def test_isometries_match_numpy(orc, B):
    rng = np.random.default_rng(B)
    blk = rng.integers(0, 1000, (B, B))
    for t in range(8):
        assert (orc_iso(orc, blk, t) == ref_iso(blk, t)).all(), t


def test_isometry_group_laws(orc):
    B = 5
    rng = np.random.default_rng(1)
    blk = rng.integers(0, 1000, (B, B))
    for t in range(8):
        cur = blk
        for _ in range(8):
            cur = orc_iso(orc, cur, t)
        assert (cur == blk).all()
    for t in (0, 2, 4, 5, 6, 7):
        assert (orc_iso(orc, orc_iso(orc, blk, t), t) == blk).all()
    assert (orc_iso(orc, orc_iso(orc, blk, 1), 3) == blk).all()
    images = [orc_iso(orc, blk, t) for t in range(8)]
    assert len({im.tobytes() for im in images}) == 8
    for a in range(8):
        for b in range(8):
            comp = orc_iso(orc, orc_iso(orc, blk, a), b)
            assert any((comp == im).all() for im in images)


def test_isometry_adjoint(orc):
    # sum r * T_t(d) == sum T_t^-1(r) * d, with t^-1 = t except 1 <-> 3
    B = 4
    rng = np.random.default_rng(2)
    r = rng.integers(0, 256, (B, B))
    d = rng.integers(0, 1021, (B, B))
    inv = [0, 3, 2, 1, 4, 5, 6, 7]
    for t in range(8):
        assert int((r * orc_iso(orc, d, t)).sum()) == int((orc_iso(orc, r, inv[t]) * d).sum())


# ---------------------------------------------------------------- search (Eq 1-3) by brute force
def brute_force_scaled(img, pool_xy, ranges_xy, B, s_num, den, rms, is_last):
    """Eq 1 evaluated per pixel for every (domain, isometry, s), scaled by
    (4 n den) to integers: e_i = 4 n den (s d_i + O - r_i) with d_i = D4/4 and
    O = mean(R) - s mean(D) (Eq 3).  Lexicographic argmin over (p, t, k)."""
    n = B * B
    s_num = np.asarray(s_num, np.int64)
    doms = []
    for v in pool_xy:
        x, y = int(v & 0xFFFF), int(v >> 16)
        d4 = ref_decimate(img[y:y + 2 * B, x:x + 2 * B])
        doms.append(np.stack([ref_iso(d4, t).ravel() for t in range(8)]))
    D = np.stack(doms)                                   # (P, 8, n)
    Sd = D[:, 0, :].sum(axis=1)                          # (P,)
    out = []
    for v in ranges_xy:
        x, y = int(v & 0xFFFF), int(v >> 16)
        r = img[y:y + B, x:x + B].astype(np.int64).ravel()
        sr = int(r.sum())
        e = (s_num[None, None, :, None] * (n * D[:, :, None, :] - Sd[:, None, None, None])
             + 4 * den * sr - 4 * n * den * r[None, None, None, :])
        E = (e * e).sum(axis=3)                          # (P, 8, S) = (4 n den)^2 E
        flat = int(np.argmin(E.ravel()))
        p, t, k = np.unravel_index(flat, E.shape)
        o = (2 * sr + n) // (2 * n)                      # round-half-up of the mean
        eq = (s_num[k] * (n * D[p, t] - Sd[p]) + 4 * n * den * o - 4 * n * den * r)
        Eq = int((eq * eq).sum())                        # (4 n den)^2 E_q
        split = (not is_last) and Eq * rms[1] ** 2 > rms[0] ** 2 * n * (4 * n * den) ** 2
        out.append((int(p), int(t), int(k), int(o), Eq, int(split), int(E.ravel()[flat])))
    return out


def check_level_against_brute(orc, img, B, L, pct, s_num, den, rms, is_last, ranges=None):
    H, W = img.shape
    pool = orc.build_pool(img, B, L, pct)
    if ranges is None:
        ranges = orc.level0_ranges(W, H, B)
    got = orc.encode_level(img, pool["xy"], ranges, B, s_num, den, rms, is_last)
    ref = brute_force_scaled(img, pool["xy"], ranges, B, s_num, den, rms, is_last)
    n = B * B
    for i, (p, t, k, o, Eq, split, _) in enumerate(ref):
        assert (got["domain"][i], got["iso"][i], got["s_idx"][i], got["offset"][i], got["split"][i]) == \
            (p, t, k, o, split), i
        # val_q = 16 den^2 n E_q and Eq here is (4 n den)^2 E_q = n * val_q
        assert n * int(got["err"][i]) == Eq, i
    return got


def test_search_fraction_brute_force_16(orc):
    """Smallest case, in exact rationals straight from Eq 1 and Eq 3."""
    img = make_image(21, 16, 16, 2)
    B, L, den = 4, 4, 16
    s_vals = [Fraction(k, den) for k in K16]
    pool = orc.build_pool(img, B, L, (3, 10))
    ranges = orc.level0_ranges(16, 16, B)
    got = orc.encode_level(img, pool["xy"], ranges, B, K16, den, (8, 1), False)
    decs = []
    for v in pool["xy"]:
        x, y = int(v & 0xFFFF), int(v >> 16)
        d = [[Fraction(int(c), 4) for c in row] for row in ref_decimate(img[y:y + 2 * B, x:x + 2 * B])]
        decs.append([ref_iso(np.array(d, dtype=object), t).ravel().tolist() for t in range(8)])
    for i, v in enumerate(ranges):
        x, y = int(v & 0xFFFF), int(v >> 16)
        r = [Fraction(int(c)) for c in img[y:y + B, x:x + B].ravel()]
        rbar = sum(r) / len(r)
        best = None
        for p, views in enumerate(decs):
            dbar = sum(views[0]) / len(r)
            for t, dv in enumerate(views):
                for k, s in enumerate(s_vals):
                    o = rbar - s * dbar                      # Eq 3
                    e = sum((s * di + o - ri) ** 2 for di, ri in zip(dv, r))   # Eq 1
                    if best is None or e < best[0]:
                        best = (e, p, t, k)
        assert (got["domain"][i], got["iso"][i], got["s_idx"][i]) == best[1:], i
        o_q = math.floor(rbar + Fraction(1, 2))
        s = s_vals[best[3]]
        dv = decs[best[1]][best[2]]
        dbar = sum(dv) / len(r)
        e_q = sum((s * (di - dbar) + o_q - ri) ** 2 for di, ri in zip(dv, r))
        assert got["offset"][i] == o_q
        assert Fraction(int(got["err"][i]), 16 * den * den * len(r)) == e_q
        assert got["split"][i] == int(e_q / len(r) > 64)


@pytest.mark.parametrize("seed,W,H,B,L,pct,s_num,den,rms", [
    (30, 32, 32, 4, 4, (3, 10), K16, 16, (8, 1)),
    (31, 32, 32, 4, 2, (0, 1), K16, 16, (5, 2)),
    (32, 48, 32, 8, 4, (3, 10), K16, 16, (8, 1)),
    (33, 32, 32, 4, 4, (3, 10), [2, 4], 10, (8, 1)),      # paper step-2 set {0.2, 0.4}
    (34, 32, 32, 2, 4, (3, 10), [5, 9], 10, (8, 1)),      # paper step-4 set {0.5, 0.9}, B = 2
    (35, 32, 32, 4, 4, (1, 2), [0, 3, 7, 10], 10, (0, 1)),
])
def test_search_scaled_brute_force(orc, seed, W, H, B, L, pct, s_num, den, rms):
    img = make_image(seed, W, H, 3)
    check_level_against_brute(orc, img, B, L, pct, s_num, den, rms, False)


def test_search_brute_force_flat_ties(orc):
    # many flat ranges: every (p, t) ties at s = 0, the lowest index must win
    img = make_image(40, 32, 32, 12)
    img[:16, :16] = 128
    check_level_against_brute(orc, img, 4, 4, (0, 1), K16, 16, (8, 1), True)


# ---------------------------------------------------------------- special cases
def test_block_constant_image(orc):
    rng = np.random.default_rng(50)
    img = np.kron(rng.integers(0, 256, (8, 8)), np.ones((8, 8), np.int64)).astype(np.uint8)
    lv = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(8, 1))
    c = lv[0]["codes"]
    assert (c["domain"] == 0).all() and (c["iso"] == 0).all() and (c["s_idx"] == 0).all()
    assert (c["err"] == 0).all() and (c["split"] == 0).all()
    assert (c["offset"] == img[::8, ::8].ravel()).all()
    assert len(lv[1]["ranges"]) == 0
    assert orc.psnr(img, orc.decode(64, 64, lv, 4)) == math.inf


def test_s_zero_split_is_rms_around_stored_mean(orc):
    img = make_image(51, 64, 64, 6)
    B, T = 8, 9
    pool = orc.build_pool(img, B, 4, (3, 10))
    ranges = orc.level0_ranges(64, 64, B)
    got = orc.encode_level(img, pool["xy"], ranges, B, [0], 16, (T, 1), False)
    for i, v in enumerate(ranges):
        x, y = int(v & 0xFFFF), int(v >> 16)
        r = img[y:y + B, x:x + B].astype(np.float64)
        o = math.floor(r.mean() + 0.5)
        assert got["offset"][i] == o
        assert got["split"][i] == int(np.mean((r - o) ** 2) > T * T)
        assert got["domain"][i] == 0 and got["iso"][i] == 0


def test_threshold_extremes(orc):
    img = make_image(52, 64, 64, 2)
    lv = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(10 ** 6, 1))
    assert lv[0]["codes"]["split"].sum() == 0 and len(lv[1]["ranges"]) == 0
    rng = np.random.default_rng(52)
    noise = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    lv = orc.encode(noise, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(0, 1))
    assert lv[0]["codes"]["split"].all() and len(lv[1]["ranges"]) == 4 * 64
    assert lv[1]["codes"]["split"].sum() == 0          # last level always accepts


# ---------------------------------------------------------------- metamorphic
def test_gray_shift(orc):
    base = (make_image(60, 64, 64, 6).astype(np.int32) * 200 // 255).astype(np.uint8)
    a = orc.encode(base, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    b = orc.encode(base + 37, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    for la, lb in zip(a, b):
        for f in ("domain", "iso", "s_idx", "split", "err"):
            assert (la["codes"][f] == lb["codes"][f]).all(), f
        assert (la["codes"]["offset"].astype(int) + 37 == lb["codes"]["offset"]).all()


def test_gray_inversion(orc):
    img = make_image(61, 64, 64, 6)
    a = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    b = orc.encode(255 - img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    for la, lb in zip(a, b):
        for f in ("domain", "iso", "s_idx", "split", "err"):
            assert (la["codes"][f] == lb["codes"][f]).all(), f
        B = la["B"]
        n = B * B
        for i, v in enumerate(la["ranges"]):
            x, y = int(v & 0xFFFF), int(v >> 16)
            sr = int(img[y:y + B, x:x + B].astype(np.int64).sum())
            half = (2 * sr) % (2 * n) == n
            assert int(lb["codes"]["offset"][i]) == 255 - int(la["codes"]["offset"][i]) + (1 if half else 0)


# ---------------------------------------------------------------- planted self-similar codes
@pytest.mark.parametrize("num,t", [(16, 0), (16, 5), (8, 3), (8, 6)])
def test_planted_zero_error_code_is_recovered(orc, num, t):
    """A range that is an exact isometric, s-scaled copy of a decimated
    domain has a zero-error code; the search must return the
    lexicographically lowest zero-error code (found here by brute force)."""
    rng = np.random.default_rng(70 + num + t)
    B, L = 4, 4
    img = rng.integers(0, 256, (32, 32)).astype(np.uint8)
    # domain at (16, 16): 2x2-constant cells with even values (so s = 1/2 stays integral)
    v = rng.integers(0, 40, (B, B)) * 2
    v[0, 0] += (-int(v.sum())) % 32      # mean of v is an even integer
    dom = np.kron(v, np.ones((2, 2), np.int64))
    img[16:24, 16:24] = dom
    vt = ref_iso(v, t) - v.mean()
    rng_rx, rng_ry = 4, 8
    planted = (vt * num // 16 + 120).astype(np.int64)
    assert planted.min() >= 0 and planted.max() <= 255
    img[rng_ry:rng_ry + B, rng_rx:rng_rx + B] = planted
    ranges = np.array([(rng_ry << 16) | rng_rx], np.uint32)
    pool = orc.build_pool(img, B, L, (0, 1))
    got = orc.encode_level(img, pool["xy"], ranges, B, K16, 16, (8, 1), True)
    ref = brute_force_scaled(img, pool["xy"], ranges, B, K16, 16, (8, 1), True)[0]
    assert ref[6] == 0                                   # a zero-error code exists
    assert int(got["err"][0]) == 0
    code = (int(got["domain"][0]), int(got["iso"][0]), int(got["s_idx"][0]))
    assert code == ref[:3]
    pidx = int(np.nonzero(pool["xy"] == ((16 << 16) | 16))[0][0])
    assert code <= (pidx, t, num)


# ---------------------------------------------------------------- decoder and Eq 4
def ref_decode(img_shape, leaves, iters, init=None):
    """Per-pixel rational decoder: pixel = clamp(O + floor(s (d - mean d) + 1/2))."""
    H, W = img_shape
    cur = np.zeros((H, W), np.int64)
    if init is not None:
        cur[:] = init
    else:
        for lf in leaves:
            cur[lf["y"]:lf["y"] + lf["B"], lf["x"]:lf["x"] + lf["B"]] = lf["O"]
    for _ in range(iters):
        nxt = cur.copy()
        for lf in leaves:
            B = lf["B"]
            d = ref_decimate(cur[lf["dy"]:lf["dy"] + 2 * B, lf["dx"]:lf["dx"] + 2 * B])
            dt = ref_iso(d, lf["t"])
            dbar = Fraction(int(d.sum()), 4 * B * B)
            s = Fraction(lf["num"], lf["den"])
            for yy in range(B):
                for xx in range(B):
                    val = lf["O"] + math.floor(s * (Fraction(int(dt[yy, xx]), 4) - dbar) + Fraction(1, 2))
                    nxt[lf["y"] + yy, lf["x"] + xx] = min(255, max(0, val))
        cur = nxt
    return cur.astype(np.uint8)


def test_decoder_matches_rational_reference(orc):
    img = make_image(80, 32, 32, 4)
    lv = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    flat = orc.leaves(lv)
    leaves = [dict(x=int(flat["lx"][i]), y=int(flat["ly"][i]), B=int(flat["lb"][i]), dx=int(flat["dx"][i]),
                   dy=int(flat["dy"][i]), t=int(flat["iso"][i]), num=int(flat["num"][i]), den=int(flat["den"][i]),
                   O=int(flat["off"][i])) for i in range(len(flat["lx"]))]
    for iters in (0, 1, 3):
        assert (orc.decode(32, 32, lv, iters) == ref_decode((32, 32), leaves, iters)).all(), iters
    # random codes exercising every isometry and negative centred values
    rng = np.random.default_rng(81)
    rand = []
    for y in range(0, 32, 8):
        for x in range(0, 32, 8):
            rand.append(dict(x=x, y=y, B=8, dx=int(rng.integers(0, 17)), dy=int(rng.integers(0, 17)),
                             t=int(rng.integers(0, 8)), num=int(rng.integers(0, 11)), den=10,
                             O=int(rng.integers(0, 256))))
    cols = {k: np.array([lf[c] for lf in rand], np.int32) for k, c in
            [("lx", "x"), ("ly", "y"), ("lb", "B"), ("dx", "dx"), ("dy", "dy"), ("iso", "t"), ("num", "num"),
             ("den", "den"), ("off", "O")]}
    for iters in (1, 4):
        assert (orc.decode_leaves(32, 32, cols, iters) == ref_decode((32, 32), rand, iters)).all()


def test_decoder_s0_gives_dc_image(orc):
    img = make_image(82, 64, 64, 4)
    lv = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=[0], s_den=16, split_rms=(8, 1))
    assert (orc.decode(64, 64, lv, 0) == orc.decode(64, 64, lv, 1)).all()


def test_decoder_is_memoryless(orc):
    img = make_image(83, 64, 64, 4)
    lv = orc.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(8, 1))
    full = orc.decode(64, 64, lv, 6)
    part = orc.decode(64, 64, lv, 2)
    assert (orc.decode(64, 64, lv, 4, init=part) == full).all()


def test_psnr_one_pixel_error(orc):
    a = np.full((40, 30), 100, np.uint8)
    b = a.copy()
    b[3, 4] = 101
    assert abs(orc.psnr(a, b) - 10 * math.log10(65025 * 40 * 30)) < 1e-12
    assert orc.psnr(a, a) == math.inf
