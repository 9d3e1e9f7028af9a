"""Pins of the oracle's contrast diagnostic (Sec. 3.2, Eq 2)."""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from paper_1502_00324_amd.synth import make_image


@pytest.fixture(scope="module")
def enc():
    img = make_image(12, 64, 64, 6)
    lv = oracle.encode(img, [(8, 4), (4, 4)], pct=(3, 10), s_num=list(range(17)), s_den=16, split_rms=(4, 1))
    return img, lv


def test_s_star_is_the_least_squares_slope(enc):
    """4 Bx / A equals numpy's least-squares slope of r on the decimated,
    isometry-mapped domain d = D4 / 4 (Eq 2)."""
    img, lv = enc
    checked = 0
    for l, v in enumerate(lv):
        B, c = v["B"], v["codes"]
        for r in range(0, len(v["ranges"]), 7):
            rxy, dxy, t = int(v["ranges"][r]), int(v["pool"]["xy"][c["domain"][r]]), int(c["iso"][r])
            bx, a = dg.bx_a(img, rxy, dxy, t, B)
            if a == 0:
                continue
            x0, y0 = rxy & 0xFFFF, rxy >> 16
            rr = img[y0:y0 + B, x0:x0 + B].astype(float).ravel()
            d = dg.chosen_view(img, dxy, t, B).astype(float).ravel() / 4.0
            slope = np.polyfit(d, rr, 1)[0]
            assert abs(4 * bx / a - slope) <= 1e-9 * max(1.0, abs(slope))
            checked += 1
    assert checked > 20


def test_decimation_and_view_against_numpy():
    rng = np.random.default_rng(3)
    blk = rng.integers(0, 256, (16, 16)).astype(np.uint8)
    np.testing.assert_array_equal(dg.decimate(blk), blk.astype(np.int64).reshape(8, 2, 8, 2).sum((1, 3)))
    img = np.zeros((16, 16), np.uint8)
    img[:, :] = blk
    d4 = dg.decimate(blk)
    # isometry 0 is the identity; 5 is the transpose (table of Sec. 2 readings)
    np.testing.assert_array_equal(dg.chosen_view(img, 0, 0, 8), d4)
    np.testing.assert_array_equal(dg.chosen_view(img, 0, 5, 8), d4.T)


def test_bins_closed_cases():
    n = 10
    assert dg.s_bin(0, 5, n) == 1                 # s* = 0: first bin
    assert dg.s_bin(-1, 5, n) == 0                # negative contrast
    assert dg.s_bin(5, 20, n) == n + 1            # 4 Bx = A: s* = 1 overflows [0, 1)
    assert dg.s_bin(4, 20, n) == 1 + 8            # s* = 0.8 -> bin 8
    assert dg.s_bin(3, 0, n) == n + 2             # flat domain


def test_a_range_copied_from_a_domain_has_unit_contrast():
    """A domain whose 2x2 cells are constant and whose decimation equals the
    range: s* = 1 exactly (overflow bin of [0, 1))."""
    rng = np.random.default_rng(5)
    r = rng.integers(0, 256, (4, 4))
    img = np.zeros((16, 16), np.uint8)
    img[0:4, 0:4] = r
    img[8:16, 8:16] = np.kron(r, np.ones((2, 2), np.int64))
    bx, a = dg.bx_a(img, 0, (8 << 16) | 8, 0, 4)
    assert a > 0 and 4 * bx == a and dg.s_bin(bx, a, 20) == 21


def test_histogram_totals(enc):
    img, lv = enc
    h = dg.s_histogram(img, lv, 16)
    for l, (v, x) in enumerate(zip(lv, h)):
        leaves = len(v["ranges"]) if l == len(lv) - 1 else int((v["codes"]["split"] == 0).sum())
        assert x["under"] + int(x["s_star"].sum()) + x["over"] + x["flat"] == leaves
        assert int(x["s_index"].sum()) == leaves
