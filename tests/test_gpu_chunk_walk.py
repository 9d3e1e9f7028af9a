"""The XCD-aware chunk walk with several chunks per workgroup, against the oracle.

The search splits the pool into chunks; with enough chunks, workgroup w runs
on XCD w % 8, the XCD's workgroups of one range group share its chunks, and
one workgroup walks G of them with one running best (the prune threshold and
the early end of a range at val 0 carry from chunk to chunk).  The default
sizes give G = 1 on images small enough for full oracle parity, so these
tests force G > 1: one partial slot per XCD (FIC_SLOTS_PER_XCD=1) and 64 KiB
chunks (FIC_CHUNK_KIB, FIC_MFMA_CHUNK_KIB).  Every matrix engine, B = 4..32,
full parity of pools and codes.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1502_00324_amd import fic
from paper_1502_00324_amd.configs import K16
from paper_1502_00324_amd.synth import make_image

pytestmark = pytest.mark.gpu
WORKERS = max(1, min(16, os.cpu_count() or 1))
MATRIX = [fic.ENGINE_MFMA, fic.ENGINE_MFMA_I8, fic.ENGINE_MFMA_F16, fic.ENGINE_MFMA_F16_16X16]
MATRIX_IDS = ["mfma", "mfma_i8", "mfma_f16", "mfma_f16_16x16"]
CHUNK_KIB = 64

# name, seed, W, H, n_rect, levels (B, L), pct, split_rms
CASES = [
    ("b8_b4_L1", 80, 256, 256, 16, [(8, 1), (4, 1)], (3, 10), (8, 1)),
    ("b32_b16_L2", 81, 256, 256, 16, [(32, 2), (16, 2)], (1, 2), (6, 1)),
]
_refs = {}


def reference(case):
    name, seed, W, H, nr, levels, pct, rms = case
    if name not in _refs:
        img = make_image(seed, W, H, nr)
        _refs[name] = (img, oracle.encode(img, levels, pct=pct, s_num=K16, s_den=16, split_rms=rms,
                                          workers=WORKERS))
    return _refs[name]


def chunks_before_rounding(engine, B, W, H, L, pct):
    """Chunks the plan cuts the expected pool into at CHUNK_KIB (before
    rounding up to a multiple of 8); with one slot per XCD a workgroup walks
    G = chunks / 8 of them, so G > 1 exactly when this is at least 9."""
    eng = fic.level_engine(engine, B)
    nd = ((W - 2 * B) // L + 1) * ((H - 2 * B) // L + 1)
    pexp = nd - (pct[0] * nd + pct[1] - 1) // pct[1]
    if eng == fic.ENGINE_MFMA_F16:   # 32x32 tiles of 32 domains, one KiB per 16-deep K-step
        form, tile, kib = fic.FORM_F16, 32, max(1, B * B // 16)
    else:                            # 16-row tiles of 16 domains
        form = fic.FORM_I8 if eng == fic.ENGINE_MFMA_I8 else fic.FORM_F16_16X16
        tile = 16
    pl, rq, dt, wpe = fic.shape_describe(form, B, 0)
    if eng != fic.ENGINE_MFMA_F16:
        kib = {1: B * B // 16, 2: 2 * (B * B // 64), 3: B * B // 32, 4: 1}[pl]
    tpc = max(8 * dt, CHUNK_KIB // kib)
    return math.ceil(math.ceil(pexp / tile) / tpc)


@pytest.mark.parametrize("engine", MATRIX, ids=MATRIX_IDS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_multi_chunk_walk_parity(monkeypatch, case, engine):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    name, seed, W, H, nr, levels, pct, rms = case
    for (B, L) in levels:
        if fic.level_engine(engine, B) != fic.ENGINE_FP32:
            assert chunks_before_rounding(engine, B, W, H, L, pct) >= 9, (B, "G would be 1")
    img, ref = reference(case)
    monkeypatch.setenv("FIC_SLOTS_PER_XCD", "1")
    monkeypatch.setenv("FIC_CHUNK_KIB", str(CHUNK_KIB))
    monkeypatch.setenv("FIC_MFMA_CHUNK_KIB", str(CHUNK_KIB))
    print("case", name, "engine", engine, flush=True)
    ctx = fic.Context(0)
    try:
        p = fic.make_params(levels, pct=pct, s_num=K16, s_den=16, split_rms=rms, engine=engine)
        pools, codes = ctx.encode([torch.from_numpy(img).cuda()], p)[0]
        torch.cuda.synchronize()
        got = fic.levels_numpy(pools, codes, p)
    finally:
        ctx.close()
    assert len(got) == len(ref)
    for l, (g, r) in enumerate(zip(got, ref)):
        for f in ("xy", "key", "sum4", "a"):
            np.testing.assert_array_equal(g["pool"][f], r["pool"][f], err_msg="%s level %d pool %s" % (name, l, f))
        np.testing.assert_array_equal(g["codes"]["xy"], r["ranges"], err_msg="%s level %d ranges" % (name, l))
        for f in ("split", "domain", "iso", "s_idx", "offset", "err"):
            np.testing.assert_array_equal(g["codes"][f], r["codes"][f], err_msg="%s level %d %s" % (name, l, f))
