"""Every compiled tile shape of every matrix form gives the oracle's codes,
and the autotuner's choice encodes like the default (the codes do not depend
on the tiling).  Inputs: seeded synthetic images (paper_1502_00324_amd.synth)."""
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
ENGINE_OF_FORM = {fic.FORM_I8: fic.ENGINE_MFMA_I8, fic.FORM_F16_16X16: fic.ENGINE_MFMA_F16_16X16,
                  fic.FORM_F16: fic.ENGINE_MFMA_F16}
# one level per block size, several domain tiles with a ragged last one
CASES = {2: (64, 48, 1), 4: (96, 64, 2), 8: (96, 64, 2), 16: (128, 96, 2), 32: (192, 128, 4)}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    c = fic.Context(0)
    yield c
    c.set_tuning({})
    c.close()


def run(ctx, img, p):
    t = torch.from_numpy(img).cuda()
    pools, codes = ctx.encode([t], p)[0]
    torch.cuda.synchronize()
    return fic.levels_numpy(pools, codes, p)


def codes_equal(got, ref, tag):
    for f in ("xy", "key", "sum4", "a"):
        np.testing.assert_array_equal(got["pool"][f], ref["pool"][f], err_msg="%s pool %s" % (tag, f))
    for f in ("domain", "iso", "s_idx", "offset", "err"):
        np.testing.assert_array_equal(got["codes"][f], ref["codes"][f], err_msg="%s %s" % (tag, f))


@pytest.mark.parametrize("form", [fic.FORM_I8, fic.FORM_F16_16X16, fic.FORM_F16], ids=list(fic.FORM_NAMES))
def test_every_tile_shape_matches_oracle(ctx, form):
    tested = 0
    for B, (W, H, L) in CASES.items():
        n = fic.shape_count(form, B)
        if n == 0:
            continue
        img = make_image(40 + B, W, H, 6)
        ref = oracle.encode(img, [(B, L)], pct=(3, 10), pool_max=0, s_num=K16, s_den=16, split_rms=(8, 1),
                            workers=WORKERS)[0]
        p = fic.make_params([(B, L)], pct=(3, 10), s_num=K16, s_den=16, split_rms=(8, 1),
                            engine=ENGINE_OF_FORM[form])
        for i in range(n):
            print("form", form, "B", B, "candidate", i, fic.shape_describe(form, B, i), flush=True)
            ctx.set_tuning({(form, B): i})
            codes_equal(run(ctx, img, p)[0], ref, "form %d B %d candidate %d" % (form, B, i))
            tested += 1
    ctx.set_tuning({})
    assert tested == sum(fic.shape_count(form, B) for B in CASES)


def test_autotune_choice_encodes_like_oracle(ctx):
    img = make_image(77, 128, 96, 10)
    levels = [(16, 2), (8, 2), (4, 2)]
    p = fic.make_params(levels, pct=(3, 10), s_num=K16, s_den=16, split_rms=(6, 1))
    t = torch.from_numpy(img).cuda()
    choice = ctx.autotune([t], p, reps=2)
    # the default engine's matrix levels: int8 planes at 16, f16 16x16 at 8, f16 32x32 at 4
    assert set(choice) >= {("mfma_i8", 16), ("mfma_f16_16x16", 8), ("mfma_f16", 4)}
    for (form, B), c in choice.items():
        assert 0 <= c < fic.shape_count(fic.FORM_NAMES.index(form), B)
    got = run(ctx, img, p)
    ref = oracle.encode(img, levels, pct=(3, 10), pool_max=0, s_num=K16, s_den=16, split_rms=(6, 1),
                        workers=WORKERS)
    for l in range(len(levels)):
        np.testing.assert_array_equal(got[l]["codes"]["xy"], ref[l]["ranges"])
        codes_equal(got[l], {"pool": ref[l]["pool"], "codes": ref[l]["codes"]}, "autotuned level %d" % l)
    ctx.set_tuning({})
