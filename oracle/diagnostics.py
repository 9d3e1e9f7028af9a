"""Contrast diagnostic (Sec. 3.2, Fig 5; Sec. 3.2.1, Fig 6) - oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  For the ranges accepted
at each level: the least-squares contrast of the chosen match (Eq 2) with
the domain decimated by 2x2 means d = D4 / 4,
    s* = (n sum r d - sum r sum d) / (n sum d^2 - (sum d)^2) = 4 Bx / A,
binned exactly over [0, 1) (underflow, nbins bins, overflow, and A = 0 where
s* is undefined), and the histogram of the chosen contrast index.
"""
from __future__ import annotations

import numpy as np

from . import iso_source


def decimate(block: np.ndarray) -> np.ndarray:
    """2x2 sums D4 of a 2B x 2B block (Sec. 2: decimated form, kept as sums)."""
    b = block.astype(np.int64)
    return b[0::2, 0::2] + b[0::2, 1::2] + b[1::2, 0::2] + b[1::2, 1::2]


def chosen_view(img: np.ndarray, dxy: int, t: int, B: int) -> np.ndarray:
    """T_t applied to the decimated domain at dxy: out[y][x] = D4[iso_source(t, y, x)]."""
    x0, y0 = dxy & 0xFFFF, dxy >> 16
    d4 = decimate(img[y0:y0 + 2 * B, x0:x0 + 2 * B])
    out = np.empty((B, B), np.int64)
    for y in range(B):
        for x in range(B):
            cy, cx = iso_source(t, B, y, x)
            out[y, x] = d4[cy, cx]
    return out


def bx_a(img: np.ndarray, rxy: int, dxy: int, t: int, B: int):
    """(Bx, A) of one range against its chosen domain and isometry."""
    x0, y0 = rxy & 0xFFFF, rxy >> 16
    r = img[y0:y0 + B, x0:x0 + B].astype(np.int64)
    d = chosen_view(img, dxy, t, B)
    n = B * B
    bx = n * int((r * d).sum()) - int(r.sum()) * int(d.sum())
    a = n * int((d * d).sum()) - int(d.sum()) ** 2
    return bx, a


def s_bin(bx: int, a: int, nbins: int) -> int:
    """Index into [under, bins..., over, flat] of s* = 4 Bx / A."""
    num = 4 * bx
    if a == 0:
        return nbins + 2
    if num < 0:
        return 0
    if num >= a:
        return nbins + 1
    return 1 + (num * nbins) // a


def s_histogram(img: np.ndarray, levels: list, nbins: int = 20) -> list:
    """levels: the oracle's encode output.  One dict per level."""
    out = []
    nl = len(levels)
    for l, lv in enumerate(levels):
        c, B = lv["codes"], lv["B"]
        keep = np.ones(len(lv["ranges"]), bool) if l == nl - 1 else (c["split"] == 0)
        hist = np.zeros(nbins + 3, np.int64)
        for r in np.nonzero(keep)[0]:
            bx, a = bx_a(img, int(lv["ranges"][r]), int(lv["pool"]["xy"][c["domain"][r]]), int(c["iso"][r]), B)
            hist[s_bin(bx, a, nbins)] += 1
        sidx = np.bincount(c["s_idx"][keep].astype(np.int64), minlength=len(lv["s_num"]))
        out.append({"under": int(hist[0]), "s_star": hist[1:nbins + 1], "over": int(hist[nbins + 1]),
                    "flat": int(hist[nbins + 2]), "s_index": sidx})
    return out
