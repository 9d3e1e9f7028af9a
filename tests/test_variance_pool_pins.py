"""Pins of the oracle's variance-keyed pool (the alternative pool the paper
cites in Sec. 1: domain blocks with small variance are deleted)."""
import math

import numpy as np
import pytest

import oracle
from paper_1502_00324_amd.synth import make_image


def test_variance_key_closed_form():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (40, 40)).astype(np.uint8)
    for (x, y, size) in [(0, 0, 8), (3, 5, 16), (10, 2, 4), (0, 0, 32)]:
        blk = img[y:y + size, x:x + size].astype(np.float64)
        m = size * size
        want = (1 << 47) - int(round(m * m * blk.var()))
        assert oracle.variance_key(img, x, y, size) == want


def brute_pool(img, B, L, pct, dn):
    """The pool rule written out with numpy variances: drop the ceil(p Nd)
    lowest-variance candidates (keep variance strictly above the c-th
    smallest), fallback to the maximum variance, then keep the DN highest
    variances (ties: lower raster index), in raster order."""
    H, W = img.shape
    nx, ny = (W - 2 * B) // L + 1, (H - 2 * B) // L + 1
    cand, var = [], []
    for iy in range(ny):
        for ix in range(nx):
            blk = img[iy * L:iy * L + 2 * B, ix * L:ix * L + 2 * B].astype(np.int64)
            m = blk.size
            var.append(int(m * (blk * blk).sum() - blk.sum() ** 2))
            cand.append(((iy * L) << 16) | (ix * L))
    var = np.array(var)
    c = math.ceil(pct[0] * len(var) / pct[1])
    if c == 0:
        keep = np.ones(len(var), bool)
    else:
        t = np.sort(var)[c - 1]
        keep = var > t
        if not keep.any():
            keep = var == var.max()
    idx = np.nonzero(keep)[0]
    if dn and len(idx) > dn:
        order = sorted(idx, key=lambda i: (-var[i], i))[:dn]
        idx = np.sort(order)
    return np.array(cand, np.uint32)[idx]


@pytest.mark.parametrize("seed,W,H,B,L,pct,dn", [
    (0, 48, 40, 4, 2, (3, 10), 0), (1, 64, 64, 8, 4, (1, 2), 0), (2, 40, 40, 4, 1, (0, 1), 25),
    (3, 64, 48, 8, 2, (3, 10), 10), (4, 32, 32, 2, 1, (9, 10), 0)])
def test_variance_pool_against_brute_force(seed, W, H, B, L, pct, dn):
    img = make_image(seed, W, H, 8)
    pool = oracle.build_pool(img, B, L, pct, dn, pool_key="variance")
    np.testing.assert_array_equal(pool["xy"], brute_pool(img, B, L, pct, dn))


def test_constant_image_keeps_every_candidate():
    img = np.full((32, 32), 77, np.uint8)
    pool = oracle.build_pool(img, 4, 2, (3, 10), 0, pool_key="variance")
    assert len(pool["xy"]) == ((32 - 8) // 2 + 1) ** 2
