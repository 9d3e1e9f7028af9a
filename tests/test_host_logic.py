"""Host logic of libfic.so on the CPU: the library is bound to a stub HIP
runtime (tests/hip_stub) in a child process, so its planning, scratch
binding, table upload, launch geometry and context life cycle run without a
GPU while no kernel executes.  The kernels themselves are covered by the GPU
parity tests."""
import json
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
STUB = os.path.join(HERE, "hip_stub")
LIB = os.path.join(ROOT, "paper_1502_00324_amd", "libfic.so")


@pytest.fixture(scope="module")
def runs(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("libfic.so is not built")
    if not shutil.which("g++") or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("no host compiler or HIP headers")
    d = tmp_path_factory.mktemp("hipstub")
    so = str(d / "libamdhip64.so.7")
    subprocess.run(["g++", "-O1", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-Wl,--version-script=" + os.path.join(STUB, "stub.map"), "-Wl,-soname,libamdhip64.so.7",
                    os.path.join(STUB, "stub.cpp"), "-o", so], check=True)
    env = dict(os.environ, LD_LIBRARY_PATH=str(d))
    r = subprocess.run([sys.executable, "-X", "faulthandler", os.path.join(STUB, "drive.py")], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


SCENARIOS = ["single_mfma", "single_fp32", "mixed_mfma_3lv", "mixed_fp32_3lv", "mixed_i8_3lv", "mixed_f16_3lv",
             "mixed_f16x_3lv",
             "mixed_b32_4lv", "large_uncapped", "large_capped",
             "paper_b2_cap", "min_images", "timing_toggle"]


@pytest.mark.parametrize("name", SCENARIOS)
def test_launch_grids_match_plans(runs, name):
    s = runs[name]
    assert all(v == 0 for v in s["status"]), s["status"]
    assert s["errors"] == []
    assert len(s["launches"]) > 0


def kinds(s):
    return [k for (k, _, _) in s["launches"]]


def test_one_launch_set_per_level(runs):
    # a batch of 8 images runs the same kernels as a batch of one
    k8, k1 = kinds(runs["mixed_mfma_3lv"]), kinds(runs["single_mfma"])
    per_rep8 = len(k8) // 2
    n8 = k8.count("k_f16_search") + k8.count("k_mfma_search")
    n1 = k1.count("k_f16_search") + k1.count("k_mfma_search")
    assert n8 == 2 * 3 and n1 == 2 * 2
    assert k8.count("k_level0") == 2
    assert per_rep8 < 120


def test_integral_images_once_per_encode(runs):
    # built by the level-0 plan only, reused by the later levels
    for name, reps in (("mixed_mfma_3lv", 2), ("single_fp32", 2), ("paper_b2_cap", 2)):
        k = kinds(runs[name])
        assert k.count("k_integ_rows") == reps and k.count("k_integ_colscan") == reps
        assert k.count("k_integ_colsum") == reps and k.count("k_integ_coladd") == reps


def test_engine_choice(runs):
    m, f = kinds(runs["mixed_mfma_3lv"]), kinds(runs["mixed_fp32_3lv"])
    i8, h = kinds(runs["mixed_i8_3lv"]), kinds(runs["mixed_f16_3lv"])
    # default: f16 32x32 tiles at B=4, f16 16x16 tiles at B=8, int8 planes at B=16
    assert "k_fp32_search" not in m and m.count("k_f16_search") == 2 and m.count("k_mfma_search") == 4
    assert runs["mixed_mfma_3lv"]["forms"] == [2, 3] * 2
    assert "k_mfma_search" not in f and "k_f16_search" not in f
    assert i8.count("k_mfma_search") == 2 * 3 and "k_f16_search" not in i8
    assert h.count("k_f16_search") == 2 * 3 and "k_mfma_search" not in h
    # the int8 engine: raw form at B=4, hi/lo planes at 8 and 16; the f16
    # 16x16 engine: plain f16 at B=8 and 16, the fused threshold at B=4
    assert runs["mixed_i8_3lv"]["forms"] == [2, 2, 1] * 2
    x = kinds(runs["mixed_f16x_3lv"])
    assert x.count("k_mfma_search") == 2 * 3 and "k_fp32_search" not in x and "k_f16_search" not in x
    assert runs["mixed_f16x_3lv"]["forms"] == [3, 3, 4] * 2
    # B=32 levels take the int8 planes form: no FP32 search in the default mix
    b32 = kinds(runs["mixed_b32_4lv"])
    assert "k_fp32_search" not in b32 and b32.count("k_f16_search") == b32.count("k_mfma_search") // 3
    assert runs["mixed_b32_4lv"]["forms"] == [2, 2, 3] * (b32.count("k_mfma_search") // 3)
    assert "k_fp32_search" not in kinds(runs["paper_b2_cap"])   # B = 2 runs on the f16 engine


def test_selection_paths(runs):
    # small levels: one fused selection launch per level, no pass launches
    for name, levels in (("single_mfma", 2), ("paper_b2_cap", 4), ("mixed_mfma_3lv", 3)):
        k = kinds(runs[name])
        assert k.count("k_sel_fused") == 2 * levels and k.count("k_sel_hist") == 0
    # large levels: 6 digit passes, 10 more with a pool-size cap
    for name, passes in (("large_uncapped", 6), ("large_capped", 16)):
        k = kinds(runs[name])
        assert k.count("k_sel_fused") == 0
        assert k.count("k_sel_hist") == passes and k.count("k_sel_pick") == passes


def test_empty_batch_and_scratch_limit(runs):
    assert runs["empty_batch"]["status"] == [0, 0] and runs["empty_batch"]["launches"] == []
    assert runs["over_limit"]["status"] == [-2] and runs["over_limit"]["launches"] == []


def test_graph_capture_and_replay(runs):
    s = runs["graphs"]
    assert all(v == 0 for v in s["status"]) and s["errors"] == []
    g = s["graph"]
    # three encodes of one argument set: one capture, then graph launches only
    assert g["first_launches"] == g["first_captured"] > 20 and g["first_replays"] == 3
    # every kernel launch of the scenario happened inside a capture; two more
    # argument sets give two more captures and graph launches
    assert len(s["launches"]) == g["captured"] and g["replays"] == 5
    # at most two graphs kept; 0 frees them
    assert g["counts"] == [1, 2, 0]


FORM_OF = {"i8": 0, "f16x": 1, "f16": 2}


def test_shape_candidates_listed(runs):
    c = runs["candidates"]
    # every matrix form has compiled shapes for its block sizes, the default first
    assert [len(c["0,%d" % B]) for B in (2, 4, 8, 16, 32)][1:] == [3, 6, 6, 3]
    assert len(c["0,2"]) == 0 and len(c["1,32"]) == 0 and len(c["2,32"]) == 0
    assert c["0,16"][0] == [2, 2, 1, 3] and c["0,32"][0] == [2, 1, 1, 2] and c["1,8"][0] == [3, 2, 12, 3]
    assert c["2,4"][0] == [0, 1, 16, 4] and all(s[0] == 4 for s in c["1,4"])
    for k, v in c.items():
        assert len({tuple(s) for s in v}) == len(v), k   # no duplicates


def test_autotune_times_every_candidate(runs):
    names = [n for n in runs if n.startswith("autotune_")]
    assert len(names) >= 12
    for name in names:
        s = runs[name]
        assert all(v == 0 for v in s["status"]) and s["errors"] == [], name
        eng, B = name.split("_")[1], int(name.split("_")[2])
        form = FORM_OF[eng]
        cands = runs["candidates"]["%d,%d" % (form, B)]
        assert {tuple(x) for x in s["shapes"]} == {tuple(x) for x in cands}, name
        # the stub's events time everything at 0: the first candidate is kept
        if len(cands) > 1:
            assert s["tuning"]["%d,%d" % (form, B)] == 0, name


def test_forced_tuning_is_used_and_validated(runs):
    s = runs["tuning_forced"]
    assert all(v == 0 for v in s["status"]) and s["errors"] == []
    c = runs["candidates"]
    assert s["shapes"] == [c["0,16"][2], c["0,8"][1], c["0,4"][0]]
    assert s["bad_set"] == -1
    after = s["after_bad"]
    assert after[0][4] == 2 and after[0][3] == 1   # the rejected call changed nothing


def test_decode_noalloc_allocates_nothing(runs):
    s = runs["decode_noalloc"]
    # status: the call, the oversized call (FIC_E_LIMIT), the ordinary decoder
    assert s["status"] == [0, -6, 0]
    n = s["noalloc"]
    # X0 per level, then 5 iterations x 2 levels, and not one allocation
    assert n["launches"] == 2 + 5 * 2 and n["allocs"] == 0
    assert n["over_launches"] == 0 and n["over_allocs"] == 0
    # the ordinary decoder grows its scratch and records timing events
    assert n["decode_allocs"] > 0


def test_launches_per_level(runs):
    # one 512 x 512 image, one level at B = 4, L = 1 (multi-pass selection):
    # selection state, keys, 6 digit passes of histogram and pick, pool
    # count, scan and scatter, moments, search-list reset, range moments,
    # operands (one launch for both sides), search queue, persistent search,
    # codes (25 launches; the last level has no child compaction)
    level = (["k_sel_init", "k_pool_keys"] + ["k_sel_hist", "k_sel_pick"] * 6 +
             ["k_bcount", "k_bscan", "k_bscatter", "k_pool_moments", "k_search_list_reset", "k_range_info", "k_prep",
              "k_search_plan", "k_f16_search", "k_finalize"])
    setup = ["k_level0", "k_integ_rows", "k_integ_colsum", "k_integ_colscan", "k_integ_coladd"]
    assert kinds(runs["large_uncapped"]) == setup + level
    # small images (one-workgroup selection), two levels: 13 launches per
    # level, plus the child compaction of the first
    small = ["k_sel_init", "k_pool_keys", "k_sel_fused", "k_bcount", "k_bscan", "k_bscatter", "k_pool_moments",
             "k_search_list_reset", "k_range_info", "k_prep", "k_search_plan", None, "k_finalize"]
    k = kinds(runs["single_mfma"])
    per_rep = len(k) // 2
    assert per_rep == len(setup) + 2 * len(small) + 3, k
    first = k[len(setup):len(setup) + len(small) + 3]
    assert [a for a, b in zip(first, small + ["k_bcount", "k_bscan", "k_bscatter"]) if b is not None and a != b] == [], first
