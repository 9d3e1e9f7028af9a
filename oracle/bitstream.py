"""Bitstream of an encoded image (Sec. 3.3, Fig 7, Eq 8) - oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain recursive
depth-first packer and unpacker, written from the paper's field list.

Per accepted range, in this order (Fig 7):
  step    2 bits   quadtree step (level) that coded the range (four steps)
  O       8 bits   stored mean of the range
  iso     3 bits   isometry
  domain  X bits   index in the level's pool list, X = ceil(log2 DN) (Eq 8)
  s       ceil(log2 |S|) bits for the level's contrast set (1 bit for two
                   values, none for one value, as in the paper's step 1)
Range addresses are not stored: records follow the regular order of the
ranges, each level-0 block in raster order and, inside a split block, its
quarters left to right and top to bottom (depth first), so the step field of
the next record tells the decoder whether the current block was split.

What the paper leaves open, and how it is read here (all bit fields MSB
first, the stream padded with zero bits to a whole byte):
  header   W (16), H (16), levels - 1 (2), log2 block0 (3); per level:
           domain step L - 1 (8), |S| - 1 (5), den - 1 (10), each num (11)
  pools    per level: DN (32), then the pool as side information (the domain
           address indexes the level's coordinate list, Sec. 3.3): mode bit
           0 = bitmap over the Nd candidates in raster order, 1 = list of
           the DN candidate indices (ascending) with ceil(log2 Nd) bits
           each; the list is used when it is strictly shorter.
"""
from __future__ import annotations

import math

import numpy as np


def ceil_log2(v: int) -> int:
    """Smallest X with 2^X >= v (Eq 8 read as the standard ceiling; 0 for v <= 1)."""
    return 0 if v <= 1 else (v - 1).bit_length()


class BitWriter:
    def __init__(self):
        self.bits = []

    def put(self, value: int, width: int):
        assert width >= 0 and 0 <= value < (1 << width) if width else value == 0, (value, width)
        for k in range(width - 1, -1, -1):
            self.bits.append((value >> k) & 1)

    def tobytes(self) -> bytes:
        b = self.bits + [0] * (-len(self.bits) % 8)
        return bytes(int("".join(map(str, b[i:i + 8])), 2) for i in range(0, len(b), 8))


class BitReader:
    def __init__(self, data: bytes):
        self.data = data
        self.pos = 0

    def get(self, width: int) -> int:
        v = 0
        for _ in range(width):
            byte = self.data[self.pos >> 3]
            v = (v << 1) | ((byte >> (7 - (self.pos & 7))) & 1)
            self.pos += 1
        return v


def n_candidates(W: int, H: int, B: int, L: int):
    return (W - 2 * B) // L + 1, (H - 2 * B) // L + 1


def pack(W: int, H: int, levels: list) -> tuple:
    """levels: the oracle's encode output (one dict per level with B, L,
    pool xy, ranges, codes, s_num, s_den).  Returns (bytes, sizes)."""
    w = BitWriter()
    nl = len(levels)
    block0 = levels[0]["B"]
    w.put(W, 16)
    w.put(H, 16)
    w.put(nl - 1, 2)
    w.put(ceil_log2(block0), 3)
    for lv in levels:
        w.put(lv["L"] - 1, 8)
        w.put(len(lv["s_num"]) - 1, 5)
        w.put(lv["s_den"] - 1, 10)
        for v in lv["s_num"]:
            w.put(int(v), 11)
    header_bits = len(w.bits)
    for lv in levels:
        nx, ny = n_candidates(W, H, lv["B"], lv["L"])
        nd = nx * ny
        xy = np.asarray(lv["pool"]["xy"], np.int64)
        dn = len(xy)
        w.put(dn, 32)
        idx = (xy >> 16) // lv["L"] * nx + (xy & 0xFFFF) // lv["L"]
        xw = ceil_log2(nd)
        if dn * xw < nd:
            w.put(1, 1)
            for i in idx:
                w.put(int(i), xw)
        else:
            w.put(0, 1)
            member = np.zeros(nd, bool)
            member[idx] = True
            for m in member:
                w.put(int(m), 1)
    pool_bits = len(w.bits) - header_bits

    # child lists: the quarters of the k-th split range of level l are
    # entries 4k..4k+3 of level l+1
    rank = [np.cumsum(lv["codes"]["split"]) - lv["codes"]["split"] for lv in levels]

    def emit(l: int, r: int):
        c = levels[l]["codes"]
        if l < nl - 1 and c["split"][r]:
            base = 4 * int(rank[l][r])
            for q in range(4):
                emit(l + 1, base + q)
            return
        lv = levels[l]
        w.put(l, 2)
        w.put(int(c["offset"][r]), 8)
        w.put(int(c["iso"][r]), 3)
        w.put(int(c["domain"][r]), ceil_log2(len(lv["pool"]["xy"])))
        w.put(int(c["s_idx"][r]), ceil_log2(len(lv["s_num"])))

    start = len(w.bits)
    for r in range(len(levels[0]["ranges"])):
        emit(0, r)
    record_bits = len(w.bits) - start
    total = len(w.bits)
    return w.tobytes(), {"header_bits": header_bits, "pool_bits": pool_bits, "record_bits": record_bits,
                         "total_bits": total}


def unpack(data: bytes) -> dict:
    """Inverse of pack: parameters, pool lists and the accepted ranges in
    stream order as (level, x, y, O, iso, domain, s_idx)."""
    rd = BitReader(data)
    W, H = rd.get(16), rd.get(16)
    nl = rd.get(2) + 1
    block0 = 1 << rd.get(3)
    levels = []
    for l in range(nl):
        L = rd.get(8) + 1
        ns = rd.get(5) + 1
        den = rd.get(10) + 1
        nums = [rd.get(11) for _ in range(ns)]
        levels.append({"B": block0 >> l, "L": L, "s_num": nums, "s_den": den})
    for lv in levels:
        nx, ny = n_candidates(W, H, lv["B"], lv["L"])
        nd = nx * ny
        dn = rd.get(32)
        if rd.get(1):
            idx = [rd.get(ceil_log2(nd)) for _ in range(dn)]
        else:
            idx = [i for i in range(nd) if rd.get(1)]
        lv["pool_xy"] = np.array([((i // nx) * lv["L"] << 16) | ((i % nx) * lv["L"]) for i in idx], np.uint32)
    recs = []

    def parse(l: int, x: int, y: int):
        save = rd.pos
        step = rd.get(2)
        rd.pos = save
        if step > l:
            h = levels[l]["B"] // 2
            for (dx, dy) in ((0, 0), (h, 0), (0, h), (h, h)):
                parse(l + 1, x + dx, y + dy)
            return
        assert step == l, "record of step %d inside a block of step %d" % (step, l)
        lv = levels[l]
        rd.get(2)
        o, iso = rd.get(8), rd.get(3)
        dom = rd.get(ceil_log2(len(lv["pool_xy"])))
        s = rd.get(ceil_log2(len(lv["s_num"])))
        recs.append((l, x, y, o, iso, dom, s))

    for y in range(0, H, block0):
        for x in range(0, W, block0):
            parse(0, x, y)
    return {"W": W, "H": H, "levels": levels, "records": recs}


def records_from_levels(levels: list) -> list:
    """The accepted ranges of an encode as (level, x, y, O, iso, domain,
    s_idx), in the depth-first stream order."""
    out = []
    nl = len(levels)
    rank = [np.cumsum(lv["codes"]["split"]) - lv["codes"]["split"] for lv in levels]

    def walk(l, r):
        c = levels[l]["codes"]
        if l < nl - 1 and c["split"][r]:
            for q in range(4):
                walk(l + 1, 4 * int(rank[l][r]) + q)
            return
        xy = int(levels[l]["ranges"][r])
        out.append((l, xy & 0xFFFF, xy >> 16, int(c["offset"][r]), int(c["iso"][r]), int(c["domain"][r]),
                    int(c["s_idx"][r])))

    for r in range(len(levels[0]["ranges"])):
        walk(0, r)
    return out


def rates(sizes: dict, W: int, H: int) -> dict:
    """Bits per pixel and compression ratio (8-bit original), with and
    without the header and pool side information."""
    px = W * H
    return {"bpp": sizes["total_bits"] / px, "bpp_records": sizes["record_bits"] / px,
            "cr": 8.0 * px / sizes["total_bits"], "cr_records": 8.0 * px / max(1, sizes["record_bits"])}
