"""The synthetic inputs are the bytes recorded in tests/golden/synth_manifest.json
(the generator's numpy PCG64 draws and FFT reproduce on this machine)."""
import json
import os

import pytest

from paper_1502_00324_amd.configs import WORKLOADS
from paper_1502_00324_amd.synth import make_image, sha256

MANIFEST = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "synth_manifest.json")))


def test_manifest_lists_every_workload():
    assert sorted(MANIFEST) == sorted(WORKLOADS)
    for name, wl in WORKLOADS.items():
        assert [(e["seed"], e["width"], e["height"], e["n_rect"]) for e in MANIFEST[name]] == list(wl.images)


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_images_match_manifest(name):
    for e in MANIFEST[name]:
        assert sha256(make_image(e["seed"], e["width"], e["height"], e["n_rect"])) == e["sha256"], (name, e["seed"])
