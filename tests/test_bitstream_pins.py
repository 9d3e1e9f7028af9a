"""Pins of the oracle's bitstream packer (Sec. 3.3, Fig 7, Eq 8).

The hand-built case below spells the expected stream bit by bit from the
field list (not from the packer), so field order, widths, bit order, the
depth-first record order and both pool encodings are fixed independently.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import bitstream as bs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.json")))


def test_eq8_address_bits_worked_value():
    g = GOLDEN["address_bits_dn64"]
    assert bs.ceil_log2(g["pool"]) == g["bits"]
    assert [bs.ceil_log2(v) for v in (1, 2, 3, 4, 5, 63, 64, 65, 1 << 20)] == [0, 1, 2, 2, 3, 6, 6, 7, 20]


def hand_levels():
    """8 x 8 image, two steps (B = 4, then 2).  Level 0: L = 4, one
    candidate; S = {1/10}.  Level 1: L = 2, 3 x 3 candidates, pool of three;
    S = {2/10, 4/10}.  The second level-0 block splits."""
    xy = lambda x, y: (y << 16) | x
    l0 = {"B": 4, "L": 4, "pool": {"xy": np.array([xy(0, 0)], np.uint32)},
          "ranges": np.array([xy(0, 0), xy(4, 0), xy(0, 4), xy(4, 4)], np.uint32),
          "codes": {"split": np.array([0, 1, 0, 0], np.uint8), "offset": np.array([10, 99, 128, 1], np.uint8),
                    "iso": np.array([3, 0, 4, 1], np.uint8), "domain": np.zeros(4, np.uint32),
                    "s_idx": np.zeros(4, np.uint8)},
          "s_num": np.array([1], np.int32), "s_den": 10}
    l1 = {"B": 2, "L": 2, "pool": {"xy": np.array([xy(0, 0), xy(4, 0), xy(0, 4)], np.uint32)},
          "ranges": np.array([xy(4, 0), xy(6, 0), xy(4, 2), xy(6, 2)], np.uint32),
          "codes": {"split": np.zeros(4, np.uint8), "offset": np.array([200, 0, 255, 17], np.uint8),
                    "iso": np.array([7, 0, 5, 2], np.uint8), "domain": np.array([2, 0, 1, 2], np.uint32),
                    "s_idx": np.array([1, 0, 1, 0], np.uint8)},
          "s_num": np.array([2, 4], np.int32), "s_den": 10}
    return [l0, l1]


HAND_BITS = "".join([
    # header: W, H, levels-1, log2 block0
    "0000000000001000", "0000000000001000", "01", "010",
    # level 0: L-1 = 3, |S|-1 = 0, den-1 = 9, num 1
    "00000011", "00000", "0000001001", "00000000001",
    # level 1: L-1 = 1, |S|-1 = 1, den-1 = 9, nums 2 and 4
    "00000001", "00001", "0000001001", "00000000010", "00000000100",
    # pool, level 0: DN = 1, Nd = 1: the list (1 x 0 bits) beats the bitmap (1 bit)
    "0" * 31 + "1", "1",
    # pool, level 1: DN = 3, Nd = 9: bitmap (9 bits) beats the list (3 x 4 bits);
    # candidates (0,0) -> 0, (4,0) -> 2, (0,4) -> 6
    "0" * 30 + "11", "0", "101000100",
    # records, depth first: step 2 | O 8 | iso 3 | domain X | s
    "00" "00001010" "011",                  # block (0,0), step 1 (level 0): X = 0, no s bit
    "01" "11001000" "111" "10" "1",         # block (4,0) split: quarter TL, X = 2, 1 s bit
    "01" "00000000" "000" "00" "0",         # TR
    "01" "11111111" "101" "01" "1",         # BL
    "01" "00010001" "010" "10" "0",         # BR
    "00" "10000000" "100",                  # block (0,4)
    "00" "00000001" "001",                  # block (4,4)
])


def to_bytes(bits):
    bits = bits + "0" * (-len(bits) % 8)
    return bytes(int(bits[i:i + 8], 2) for i in range(0, len(bits), 8))


def test_hand_built_stream_bit_by_bit():
    data, sizes = bs.pack(8, 8, hand_levels())
    assert data == to_bytes(HAND_BITS)
    assert sizes["total_bits"] == len(HAND_BITS)
    assert sizes["record_bits"] == 13 + 4 * 16 + 2 * 13
    assert sizes["header_bits"] == 37 + (8 + 5 + 10 + 11) + (8 + 5 + 10 + 22)


def test_hand_built_stream_unpacks():
    u = bs.unpack(to_bytes(HAND_BITS))
    assert (u["W"], u["H"]) == (8, 8)
    assert [(lv["B"], lv["L"], lv["s_num"], lv["s_den"]) for lv in u["levels"]] == [(4, 4, [1], 10), (2, 2, [2, 4], 10)]
    assert list(u["levels"][1]["pool_xy"]) == [0, 4, 4 << 16]
    assert u["records"] == [(0, 0, 0, 10, 3, 0, 0), (1, 4, 0, 200, 7, 2, 1), (1, 6, 0, 0, 0, 0, 0),
                            (1, 4, 2, 255, 5, 1, 1), (1, 6, 2, 17, 2, 2, 0), (0, 0, 4, 128, 4, 0, 0),
                            (0, 4, 4, 1, 1, 0, 0)]


def test_paper_field_widths():
    g = GOLDEN["code_field_bits"]
    # the paper's schedule: one s value at step 1, two at steps 2-4, DN = 64
    assert bs.ceil_log2(1) == g["s_step_1"] and bs.ceil_log2(2) == g["s_steps_2_to_4"]
    assert g["step"] + g["offset"] + g["iso"] + bs.ceil_log2(64) + g["s_step_1"] == 19


@pytest.fixture(scope="module")
def encodes():
    from paper_1502_00324_amd.synth import make_image
    out = []
    for seed, W, H, levels, pct, dn, s_num, s_den in [
            (3, 64, 64, [(8, 4), (4, 4)], (3, 10), 0, list(range(17)), 16),
            (4, 64, 48, [(16, 4), (8, 4), (4, 4), (2, 4)], (0, 1), 20, ((1,), (2, 4), (3, 8), (5, 9)), 10),
            (5, 96, 64, [(8, 2), (4, 2)], (1, 2), 0, (0, 3, 7, 10), 10)]:
        img = make_image(seed, W, H, 6)
        lv = oracle.encode(img, levels, pct=pct, pool_max=dn, s_num=s_num, s_den=s_den, split_rms=(4, 1))
        out.append((img, lv))
    return out


def test_record_bits_closed_form(encodes):
    for img, lv in encodes:
        H, W = img.shape
        _, sizes = bs.pack(W, H, lv)
        want = 0
        for l, v in enumerate(lv):
            leaves = len(v["ranges"]) if l == len(lv) - 1 else int((v["codes"]["split"] == 0).sum())
            want += leaves * (2 + 8 + 3 + bs.ceil_log2(len(v["pool"]["xy"])) + bs.ceil_log2(len(v["s_num"])))
        assert sizes["record_bits"] == want


def test_round_trip(encodes):
    for img, lv in encodes:
        H, W = img.shape
        data, sizes = bs.pack(W, H, lv)
        assert len(data) == (sizes["total_bits"] + 7) // 8
        u = bs.unpack(data)
        assert u["records"] == bs.records_from_levels(lv)
        for a, b in zip(u["levels"], lv):
            np.testing.assert_array_equal(a["pool_xy"], b["pool"]["xy"])
            assert list(a["s_num"]) == list(b["s_num"]) and a["s_den"] == b["s_den"] and a["L"] == b["L"]
        # the leaves tile the image exactly once
        cover = np.zeros((H, W), int)
        for (l, x, y, *_rest) in u["records"]:
            B = lv[l]["B"]
            cover[y:y + B, x:x + B] += 1
        assert (cover == 1).all()
