"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol include/fic.h declares, validates arguments on the host, and its
independently generated entropy table equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1502_00324_amd import fic
from paper_1502_00324_amd.configs import WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fic_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fic.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fic.EXPORTED)


def test_entropy_table_matches_oracle(orc):
    assert (fic.entropy_table() == orc.entropy_table()).all()


def test_strerror():
    assert fic.strerror(fic.FIC_OK) == "ok"
    for st in (fic.FIC_E_INVALID, fic.FIC_E_NOMEM, fic.FIC_E_HIP, fic.FIC_E_CAPACITY, fic.FIC_E_ARCH, fic.FIC_E_LIMIT):
        assert fic.strerror(st) not in ("ok", "unknown status")


def preset_params(wl):
    return fic.make_params(wl.levels, pct=wl.pct, pool_max=wl.pool_max, s_num=wl.s_num, s_den=wl.s_den,
                           split_rms=wl.split_rms)


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_presets_validate(name):
    wl = WORKLOADS[name]
    p = preset_params(wl)
    for (_, W, H, _) in wl.images:
        assert fic.validate_params(p, W, H) == fic.FIC_OK, (name, W, H)


BAD = [
    ("levels0", lambda p: setattr(p, "levels", 0)),
    ("levels5", lambda p: setattr(p, "levels", 5)),
    ("block0_not_pow2", lambda p: setattr(p, "block0", 12)),
    ("block0_64", lambda p: setattr(p, "block0", 64)),
    ("last_block_1", lambda p: (setattr(p, "block0", 4), setattr(p, "levels", 3))),
    ("step0", lambda p: p.step.__setitem__(1, 0)),
    ("pct_ge_1", lambda p: setattr(p, "pool_pct", fic.Ratio(1, 1))),
    ("pct_den0", lambda p: setattr(p, "pool_pct", fic.Ratio(0, 0))),
    ("pool_max_neg", lambda p: setattr(p, "pool_max", -1)),
    ("s_count0", lambda p: p.s_count.__setitem__(0, 0)),
    ("s_count33", lambda p: p.s_count.__setitem__(0, 33)),
    ("s_den0", lambda p: p.s_den.__setitem__(0, 0)),
    ("s_den1025", lambda p: p.s_den.__setitem__(0, 1025)),
    ("s_not_ascending", lambda p: (p.s_num[1].__setitem__(3, 2))),
    ("s_above_den", lambda p: (p.s_num[2].__setitem__(16, 17))),
    ("s_negative", lambda p: (p.s_num[0].__setitem__(0, -1))),
    ("rms_den0", lambda p: p.split_rms.__setitem__(0, fic.Ratio(8, 0))),
    ("rms_den17", lambda p: p.split_rms.__setitem__(0, fic.Ratio(8, 17))),
    ("rms_neg", lambda p: p.split_rms.__setitem__(0, fic.Ratio(-1, 1))),
    ("engine5", lambda p: setattr(p, "engine", 5)),
    ("pool_key2", lambda p: setattr(p, "pool_key", 2)),
    ("pool_key_neg", lambda p: setattr(p, "pool_key", -1)),
    ("engine_neg", lambda p: setattr(p, "engine", -1)),
]


@pytest.mark.parametrize("name,mut", BAD, ids=[b[0] for b in BAD])
def test_validate_rejects(name, mut):
    p = preset_params(WORKLOADS["c2_512"])
    mut(p)
    assert fic.validate_params(p, 512, 512) == fic.FIC_E_INVALID


@pytest.mark.parametrize("W,H", [(500, 512), (512, 24), (16, 512), (70000, 64)])
def test_validate_rejects_geometry(W, H):
    assert fic.validate_params(preset_params(WORKLOADS["c2_512"]), W, H) == fic.FIC_E_INVALID


def test_query_capacity_counts():
    p = preset_params(WORKLOADS["c2_512"])
    pc, rc = fic.query_capacity(p, 512, 512)
    # candidates ((N - 2B)/L + 1)^2; 15625 at B = 8, L = 4 is the worked example of Sec. 2
    assert pc == [121 ** 2, 15625, 127 ** 2]
    assert rc == [32 ** 2, 64 ** 2, 128 ** 2]
    p.pool_max = 64
    pc, _ = fic.query_capacity(p, 512, 512)
    assert pc == [64, 64, 64]


def test_null_context_is_rejected_before_any_device_work():
    L = fic.lib()
    p = preset_params(WORKLOADS["c1_64"])
    img = fic.Image(None, 64, 64, 64)
    pool = fic.PoolC()
    codes = fic.CodesC()
    assert L.fic_encode(None, ctypes.byref(img), 1, ctypes.byref(p), ctypes.byref(pool), ctypes.byref(codes),
                        None) == fic.FIC_E_INVALID
    assert L.fic_build_domain_pool(None, ctypes.byref(img), 8, 4, fic.Ratio(3, 10), 0, 0, ctypes.byref(pool),
                                   None) == fic.FIC_E_INVALID
    assert L.fic_decode(None, ctypes.byref(p), ctypes.byref(pool), ctypes.byref(codes), 64, 64, 1, None,
                        None) == fic.FIC_E_INVALID
    assert L.fic_ctx_set_scratch_limit(None, 0) == fic.FIC_E_INVALID


def test_ctx_create_reports_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert fic.lib().fic_ctx_create(ctypes.byref(h), 0) == fic.FIC_E_HIP
    assert not h.value


def test_shape_queries_are_host_only():
    assert fic.shape_count(fic.FORM_I8, 16) == 6 and fic.shape_count(fic.FORM_F16, 32) == 0
    assert fic.shape_count(fic.FORM_I8, 12) == 0 and fic.lib().fic_shape_count(7, 8) == 0
    assert fic.shape_describe(fic.FORM_F16_16X16, 8, 0) == (3, 2, 12, 3)
    with pytest.raises(fic.FicError):
        fic.shape_describe(fic.FORM_I8, 8, 99)
    assert fic.lib().fic_ctx_set_tuning(None, None) == fic.FIC_E_INVALID


def test_level_engine_resolution():
    M, F, I8, H = fic.ENGINE_MFMA, fic.ENGINE_FP32, fic.ENGINE_MFMA_I8, fic.ENGINE_MFMA_F16
    X = fic.ENGINE_MFMA_F16_16X16
    assert [fic.level_engine(M, B) for B in (2, 4, 8, 16, 32)] == [H, H, X, I8, I8]
    assert [fic.level_engine(I8, B) for B in (2, 4, 8, 16, 32)] == [F, I8, I8, I8, I8]
    assert [fic.level_engine(H, B) for B in (2, 4, 8, 16, 32)] == [H, H, H, H, F]
    assert [fic.level_engine(X, B) for B in (2, 4, 8, 16, 32)] == [X, X, X, X, F]
    assert all(fic.level_engine(F, B) == F for B in (2, 4, 8, 16, 32))
    assert fic.lib().fic_level_engine(5, 8) == fic.FIC_E_INVALID
    assert fic.lib().fic_level_engine(M, 12) == fic.FIC_E_INVALID
    assert fic.lib().fic_level_engine(M, 64) == fic.FIC_E_INVALID
