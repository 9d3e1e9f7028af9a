"""The encoder oracle: plain exact CPU implementation of the paper's method.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke() check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
loads it and shares no code with it.

The arithmetic lives in fic_oracle.c (plain nested loops, int64); this
module marshals numpy arrays and drives the quadtree steps (Sec. 2, Fig 1):
level 0 is every B x B range in raster order, level l+1 holds the four
quarters of every range that level l split, in parent order, each as
top-left, top-right, bottom-left, bottom-right.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "fic_oracle.c")


def build(force: bool = False) -> str:
    """Compile fic_oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-Wall", "-Wextra",
                               "-o", tmp, SRC_PATH], cwd=HERE)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.orc_entropy_table.argtypes = [P, i32]
        L.orc_entropy_key.argtypes = [P, i32, i32, i32, i32]
        L.orc_entropy_key.restype = i64
        L.orc_candidates.argtypes = [i32, i32, i32, i32, P, i32]
        L.orc_build_pool.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32, i32, P, P, P, P, i32, i32]
        L.orc_variance_key.argtypes = [P, i32, i32, i32, i32]
        L.orc_variance_key.restype = i64
        L.orc_iso_source.argtypes = [i32, i32, i32, i32, P, P]
        L.orc_encode_level.argtypes = [P, i32, i32, i32, P, i32, P, i32, i32, P, i32, i32, i32, i32, i32,
                                       P, P, P, P, P, P, i32]
        L.orc_decode.argtypes = [i32, i32, i32] + [P] * 9 + [i32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def entropy_table() -> np.ndarray:
    out = np.zeros(4097, np.int64)
    assert lib().orc_entropy_table(_p(out), 4097) == 0
    return out


def entropy_key(img: np.ndarray, x: int, y: int, size: int) -> int:
    img = np.ascontiguousarray(img, np.uint8)
    return int(lib().orc_entropy_key(_p(img), img.shape[1], x, y, size))


def candidates(W: int, H: int, B: int, L: int) -> np.ndarray:
    n = lib().orc_candidates(W, H, B, L, None, 0)
    if n < 0:
        raise ValueError("invalid candidate geometry")
    out = np.zeros(n, np.uint32)
    lib().orc_candidates(W, H, B, L, _p(out), n)
    return out


def iso_source(t: int, B: int, y: int, x: int):
    sy, sx = ctypes.c_int(), ctypes.c_int()
    lib().orc_iso_source(t, B, y, x, ctypes.byref(sy), ctypes.byref(sx))
    return sy.value, sx.value


POOL_KEYS = {"entropy": 0, "variance": 1}


def variance_key(img: np.ndarray, x: int, y: int, size: int) -> int:
    img = np.ascontiguousarray(img, np.uint8)
    return lib().orc_variance_key(_p(img), img.shape[1], x, y, size)


def build_pool(img: np.ndarray, B: int, L: int, pct=(0, 1), pool_max: int = 0, pool_key: str = "entropy",
               threads: int = 1) -> dict:
    """Sec. 3 Eq 5-6 (entropy key) or the variance key of the cited
    alternative; the same percentile and DN rules for both.  threads: the
    candidate keys are split over that many threads (same values)."""
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    nd = lib().orc_candidates(W, H, B, L, None, 0)
    if nd < 0:
        raise ValueError("invalid candidate geometry")
    xy = np.zeros(nd, np.uint32)
    key = np.zeros(nd, np.int64)
    sum4 = np.zeros(nd, np.uint32)
    a = np.zeros(nd, np.int64)
    cnt = lib().orc_build_pool(_p(img), W, H, W, B, L, pct[0], pct[1], pool_max, POOL_KEYS[pool_key],
                               _p(xy), _p(key), _p(sum4), _p(a), nd, max(1, min(64, int(threads))))
    if cnt < 0:
        raise ValueError("orc_build_pool failed: %d" % cnt)
    return {"xy": xy[:cnt].copy(), "key": key[:cnt].copy(), "sum4": sum4[:cnt].copy(), "a": a[:cnt].copy(),
            "candidates": nd}


def level0_ranges(W: int, H: int, B: int) -> np.ndarray:
    ys, xs = np.meshgrid(np.arange(0, H, B), np.arange(0, W, B), indexing="ij")
    return ((ys.astype(np.uint32) << 16) | xs.astype(np.uint32)).ravel()


def children(ranges_xy: np.ndarray, split: np.ndarray, B: int) -> np.ndarray:
    """Quarters of every split range, parent order, TL, TR, BL, BR."""
    h = B // 2
    out = []
    for xy, s in zip(ranges_xy.tolist(), split.tolist()):
        if s:
            x, y = xy & 0xFFFF, xy >> 16
            out += [(y << 16) | x, (y << 16) | (x + h), ((y + h) << 16) | x, ((y + h) << 16) | (x + h)]
    return np.array(out, np.uint32)


def encode_level(img: np.ndarray, pool_xy: np.ndarray, ranges_xy: np.ndarray, B: int,
                 s_num, s_den: int, split_rms=(8, 1), is_last: bool = False, workers: int = 1) -> dict:
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    pool_xy = np.ascontiguousarray(pool_xy, np.uint32)
    ranges_xy = np.ascontiguousarray(ranges_xy, np.uint32)
    s_num = np.ascontiguousarray(s_num, np.int32)
    R = len(ranges_xy)
    out = {"split": np.zeros(R, np.uint8), "domain": np.zeros(R, np.uint32), "iso": np.zeros(R, np.uint8),
           "s_idx": np.zeros(R, np.uint8), "offset": np.zeros(R, np.uint8), "err": np.zeros(R, np.int64)}
    if R == 0:
        return out

    # workers: threads in the C search, each over a slice of the ranges
    st = lib().orc_encode_level(_p(img), W, H, W, _p(pool_xy), len(pool_xy), _p(ranges_xy), R, B,
                                _p(s_num), len(s_num), s_den, split_rms[0], split_rms[1], int(is_last),
                                *(_p(out[k]) for k in ("split", "domain", "iso", "s_idx", "offset", "err")),
                                max(1, min(64, int(workers))))
    if st != 0:
        raise ValueError("orc_encode_level failed: %d" % st)
    return out


def encode(img: np.ndarray, levels, pct=(3, 10), pool_max: int = 0, s_num=None, s_den: int = 16,
           split_rms=None, workers: int = 1, pool_key: str = "entropy") -> list:
    """Whole quadtree.  levels: list of (B, L) per step.  s_num / s_den /
    split_rms may be per-level lists or single values.  Returns one dict
    per level with the pool, the ranges and the codes."""
    H, W = img.shape
    nl = len(levels)
    s_num_l = s_num if (s_num is not None and isinstance(s_num[0], (list, tuple, np.ndarray))) else [s_num] * nl
    s_den_l = s_den if isinstance(s_den, (list, tuple)) else [s_den] * nl
    rms_l = split_rms if (split_rms is not None and isinstance(split_rms[0], (list, tuple))) else [split_rms] * nl
    out = []
    ranges = level0_ranges(W, H, levels[0][0])
    for li, (B, L) in enumerate(levels):
        pool = build_pool(img, B, L, pct, pool_max, pool_key, threads=workers)
        is_last = li == nl - 1
        codes = encode_level(img, pool["xy"], ranges, B, s_num_l[li], s_den_l[li],
                             rms_l[li] if rms_l[li] is not None else (0, 1), is_last, workers)
        out.append({"B": B, "L": L, "pool": pool, "ranges": ranges, "codes": codes,
                    "s_num": np.asarray(s_num_l[li], np.int32), "s_den": s_den_l[li]})
        if not is_last:
            ranges = children(ranges, codes["split"], B)
    return out


def leaves(levels: list) -> dict:
    """Accepted ranges of every level as flat arrays for the decoder."""
    cols = {k: [] for k in ("lx", "ly", "lb", "dx", "dy", "iso", "num", "den", "off")}
    for lv in levels:
        c, B = lv["codes"], lv["B"]
        keep = c["split"] == 0
        rxy = lv["ranges"][keep]
        dxy = lv["pool"]["xy"][c["domain"][keep]]
        cols["lx"].append(rxy & 0xFFFF)
        cols["ly"].append(rxy >> 16)
        cols["lb"].append(np.full(len(rxy), B))
        cols["dx"].append(dxy & 0xFFFF)
        cols["dy"].append(dxy >> 16)
        cols["iso"].append(c["iso"][keep])
        cols["num"].append(lv["s_num"][c["s_idx"][keep]])
        cols["den"].append(np.full(len(rxy), lv["s_den"]))
        cols["off"].append(c["offset"][keep])
    return {k: np.ascontiguousarray(np.concatenate(v) if v else np.zeros(0), np.int32) for k, v in cols.items()}


def decode(W: int, H: int, levels: list, iters: int, init: np.ndarray | None = None) -> np.ndarray:
    return decode_leaves(W, H, leaves(levels), iters, init)


def decode_leaves(W: int, H: int, lv: dict, iters: int, init: np.ndarray | None = None) -> np.ndarray:
    out = np.zeros((H, W), np.uint8)
    init_p = None
    if init is not None:
        init = np.ascontiguousarray(init, np.uint8)
        assert init.shape == (H, W)
        init_p = _p(init)
    st = lib().orc_decode(W, H, len(lv["lx"]), *(_p(lv[k]) for k in ("lx", "ly", "lb", "dx", "dy", "iso",
                                                                     "num", "den", "off")), iters, init_p, _p(out))
    if st != 0:
        raise ValueError("orc_decode failed: %d" % st)
    return out


def sse(a: np.ndarray, b: np.ndarray) -> int:
    d = a.astype(np.int64) - b.astype(np.int64)
    return int((d * d).sum())


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    """Eq 4: 10 log10(255^2 / MSE); +inf for identical images."""
    e = sse(a, b)
    return math.inf if e == 0 else 10.0 * math.log10(65025.0 * a.size / e)
